"""Parity at the largest size: A 200000 x 500000 (4 N(0,1) nonzeros per
column), FP64, B = 512.

* Bound tightening at a fixed iteration count, default options (the tile
  autotuner times its candidate shapes on the first block of iterations), 65
  iterations (one full evaluation with its restart tests).
* The strong-branching batch of the benchmark line, converged, in the
  options the benchmark times (its command line's defaults): the base LP
  solved on the GPU, 512 bound changes on 256 fractional variables of its
  root, warm start from it, C = 18 with stopping tests every 6 iterations,
  tolerance 1e-4, captured blocks of iterations, results written into the
  caller's device tensors.

The oracle recomputes a sample of the LPs one at a time with the same step
size and start; every LP of the batch must also be finite and still running
or stopped with a valid status."""
import numpy as np
import pytest

import bench
import oracle as O
from tests.gpu_common import make_ctx, lp_for, assert_trajectory_match
from tests.gpu_common import oracle_run
from workloads import make_cfg5, obbt_deltas, choose_vars, choose_fractional, fsb_deltas, \
    seed_for, deltas, BASE

pytestmark = pytest.mark.gpu

K = 65
LINE = bench.make_parser().parse_args([])


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


def test_largest_size_sampled_lps_match_oracle(P):
    inst = make_cfg5()
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(inst.n, 256, seed=512))
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=0.0, max_iters=K)
        st = ctx.get_batch(want_x=False, want_y=False)
        sample = [0, 255, 256, 511]
        res = {j: (ctx.get(j), ctx.get_trace(j)) for j in sample}
    assert np.all(st["iters"] == K) and np.all(st["status"] == P.STATUS_ITERATION_LIMIT)
    assert np.all(np.isfinite(st["kkt"]))
    for j in sample:
        ores = O.solve(lp_for(lp, D[j]), O.Options(tol=0.0, max_iters=K, step_size=eta))
        assert_trajectory_match(*res[j], ores, what=f"LP {j}")


@pytest.fixture(scope="module")
def line_root(P):
    """The line's base LP solved on the GPU (FP64, C = 24) and draw 0 of its
    candidates."""
    inst = make_cfg5(base=0)
    lp = O.from_instance(inst)
    with P.Context.from_instance(inst, eval_every=LINE.cfg5_root_eval, max_batch=1) as ctx:
        eta, _ = ctx.step_size
        ctx.set_batch(deltas([BASE], [0], [0.0]))
        ctx.solve(tol=1e-6, max_iters=200000)
        root = ctx.get(0)
        w = ctx.get_trace(0)["w"]
    assert root["status"] == P.STATUS_OPTIMAL
    D = fsb_deltas(root["x"], choose_fractional(root["x"], LINE.cfg5_vars,
                                                seed_for(5, LINE.cfg5_draw_seed)))
    return inst, lp, eta, root, w, D


def test_mixed32_line_points_meet_tolerance_against_a(P, line_root):
    """Draw 0 of the line with FP32 iterates and products (FP64 sums): every
    LP it reports optimal has an FP64 twin within 1e-7 in objective, and the
    oracle measures a sample of its points within the tolerance against the
    true A (the FP32 run multiplies by A rounded to FP32)."""
    inst, lp, eta, root, w, D = line_root
    res = {}
    for prec in (P.FP64, P.MIXED32):
        with P.Context.from_instance(inst, eval_every=LINE.cfg5_eval,
                                     stop_every=LINE.cfg5_stop_every, max_batch=512,
                                     step_size=eta, precision=prec) as ctx:
            ctx.set_batch(D, x_warm=root["x"], y_warm=root["y"], w_warm=np.full(len(D), w))
            ctx.solve(tol=1e-4, max_iters=LINE.cfg5_mixed_iters)
            res[prec] = ctx.get_batch()
    a, b = res[P.FP64], res[P.MIXED32]
    both = (a["status"] == P.STATUS_OPTIMAL) & (b["status"] == P.STATUS_OPTIMAL)
    assert both.sum() >= len(D) - 4
    err = np.abs(b["obj"][both] - a["obj"][both]) / (1 + np.abs(a["obj"][both]))
    rel = []
    order = np.argsort(b["iters"], kind="stable")
    for j in [int(order[k]) for k in np.linspace(0, len(order) - 1, 8).astype(int)]:
        if b["status"][j] == P.STATUS_OPTIMAL:
            rel.append(O.kkt(lp_for(lp, D[j]), b["X"][j], b["Y"][j]).rel)
    print(f"MIXED32 line: objective difference max {err.max():.2e}; oracle KKT of FP32 points "
          f"against A: max {max(rel):.2e} over {len(rel)} LPs")
    assert err.max() <= 1e-7
    assert rel and max(rel) <= 1e-4


def test_strong_branching_line_sampled_lps_match_oracle(P, line_root):
    """Draw 0 of the benchmark line: the first LP of the batch, the LP at the
    three-quarter point of the iteration counts and the slowest LP follow the
    oracle's trajectories from the same root (statuses, iteration counts,
    restart logs, iterates and KKT measures), and solved alone they give the
    batch's bits (the batch's last LPs run in narrow storage).  The batch
    writes its results into device tensors of the caller, as the benchmark
    does; each read of them gives the same bits.

    Per coordinate the iterates are compared on the scale max(|o_i|, rms(o), 1)
    (elem_scale): after hundreds of iterations on duals whose entries are in
    the thousands (rms 1765 for the slowest LP), a dual entry near zero carries
    the rounding of the terms mixed into it, e.g. 4.1e-9 on an entry of 0.58,
    2.3e-12 of the vector's scale; the norm-relative check stays at 1e-9."""
    import torch
    inst, lp, eta, root, w, D = line_root
    C, S = LINE.cfg5_eval, LINE.cfg5_stop_every
    assert len(D) == 512
    dev = torch.device("cuda:0")
    X = torch.full((len(D), inst.n), float("nan"), dtype=torch.float64, device=dev)
    Y = torch.full((len(D), inst.m), float("nan"), dtype=torch.float64, device=dev)
    with P.Context.from_instance(inst, eval_every=C, stop_every=S, max_batch=512,
                                 step_size=eta, use_graphs=LINE.graphs) as ctx:
        ctx.set_result_buffers(X, Y, len(D))
        ctx.set_batch(D, x_warm=root["x"], y_warm=root["y"], w_warm=np.full(len(D), w))
        ctx.solve(tol=1e-4, max_iters=100000)
        st = ctx.get_batch(X=X, Y=Y, mem=P.MEM_DEVICE)
        order = np.argsort(st["iters"], kind="stable")
        sample = sorted({0, int(order[3 * len(order) // 4]), int(order[-1])})
        res = {j: (ctx.get(j), ctx.get_trace(j)) for j in sample}
    for j in sample:
        assert np.array_equal(X[j].cpu().numpy(), res[j][0]["x"]), j
        assert np.array_equal(Y[j].cpu().numpy(), res[j][0]["y"]), j
    assert not torch.isnan(X).any().item() and not torch.isnan(Y).any().item()
    # the same LPs alone (one column, never moved to narrow storage): the same
    # bits as in the batch, whose last LPs ran in blocks of stride 16
    with P.Context.from_instance(inst, eval_every=C, stop_every=S, max_batch=1,
                                 step_size=eta) as one:
        for j in sample:
            one.set_batch(D[j:j + 1], x_warm=root["x"], y_warm=root["y"], w_warm=np.full(1, w))
            one.solve(tol=1e-4, max_iters=100000)
            g, tr = one.get(0), one.get_trace(0)
            assert g["status"] == res[j][0]["status"] and g["iters"] == res[j][0]["iters"], j
            assert tr["restart_log"] == res[j][1]["restart_log"], j
            for key in ("x", "y"):
                assert np.array_equal(g[key], res[j][0][key]), (j, key)
            for key in ("x_iter", "y_iter"):
                assert np.array_equal(tr[key], res[j][1][key]), (j, key)
    ok = np.isin(st["status"], [P.STATUS_OPTIMAL, P.STATUS_PRIMAL_INFEASIBLE])
    assert np.all(ok), np.bincount(st["status"])
    assert np.all(st["kkt"][st["status"] == P.STATUS_OPTIMAL, 3] <= 1e-4)
    for j in sample:
        ores = oracle_run(lp_for(lp, D[j]), eta, 1e-4, 100000, root["x"], root["y"], w,
                          eval_every=C, stop_every=S)
        print("LP", j, "iters", res[j][0]["iters"], "restarts", res[j][1]["restart_log"][:8])
        assert_trajectory_match(*res[j], ores, what=f"line LP {j}", floor="rms")


def test_repeated_line_solves_replay_the_same_bits(P, line_root):
    """One context solves three draws of the line, then the first again, in
    the benchmark's options (captured blocks, results in the caller's
    tensors): its captured blocks of iterations are replayed across solves
    and across the narrow strides the last LPs move through (16, 4, 2, 1),
    and every solve gives the statuses, iteration counts, KKT measures,
    objectives and result rows of the same draw solved without graphs into
    the context's own blocks."""
    import torch
    inst, lp, eta, root, w, D0 = line_root
    draws = [D0] + [fsb_deltas(root["x"], choose_fractional(
        root["x"], LINE.cfg5_vars, seed_for(5, LINE.cfg5_draw_seed + r))) for r in (1, 2)]
    B = len(D0)
    dev = torch.device("cuda:0")
    X = torch.empty((B, inst.n), dtype=torch.float64, device=dev)
    Y = torch.empty((B, inst.m), dtype=torch.float64, device=dev)
    rows = [0, B // 2, B - 1]
    got = {}
    for graphs, seq in ((1, [0, 1, 2, 0]), (0, [0, 1, 2])):
        with P.Context.from_instance(inst, eval_every=LINE.cfg5_eval,
                                     stop_every=LINE.cfg5_stop_every, max_batch=B,
                                     step_size=eta, use_graphs=graphs) as ctx:
            if graphs:
                ctx.set_result_buffers(X, Y, B)
            for k, i in enumerate(seq):
                ctx.set_batch(draws[i], x_warm=root["x"], y_warm=root["y"], w_warm=np.full(B, w))
                ctx.solve(tol=1e-4, max_iters=100000)
                st = ctx.get_batch(want_x=False, want_y=False)
                st["rows"] = [(ctx.get(j)["x"], ctx.get(j)["y"]) for j in rows]
                if graphs:
                    st["ext"] = [(X[j].cpu().numpy(), Y[j].cpu().numpy()) for j in rows]
                got[(graphs, k, i)] = st
    for (graphs, k, i), st in got.items():
        ref = got[(0, i, i)]
        for key in ("status", "iters", "kkt", "obj"):
            assert np.array_equal(st[key], ref[key], equal_nan=True), (graphs, k, i, key)
        for r, (a, b) in enumerate(zip(st["rows"], ref["rows"])):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (graphs, k, i, r)
        for r, (a, b) in enumerate(zip(st.get("ext", ()), ref["rows"])):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (graphs, k, i, r)
