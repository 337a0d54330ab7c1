"""GPU path vs the FP64 reference solver, through the C ABI.

Tolerances: FP64 iterates after a fixed number of iterations agree to 1e-9
relative (per LP, ||z_gpu - z_ref|| / max(||z_ref||, 1)), with identical
statuses, iteration counts and restart iterations; converged runs reach
1e-4 relative KKT with objectives within 4e-4 (1 + |obj|), the bracket two
1e-4-optimal points leave by the gap test of eq:stopping.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_common import (ITER_RTOL, rel_err, elem_err, lp_for, make_ctx, cfg2_setup, oracle_run,
                              assert_trajectory_match)
from workloads import (make_cfg1, make_cfg2, make_cfg3, make_tiny, obbt_deltas, choose_vars,
                       deltas, BASE, SET_LO, SET_HI, OBJ_UNIT)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


# ---------------------------------------------------------------------------
# single LP (B = 1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K", [1, 2, 10, 64, 65, 66, 100, 1000, 3000])
def test_cfg1_fixed_iterations(P, K):
    inst = make_cfg1()
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    ores = oracle_run(lp, eta, 0.0, K)
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(deltas([BASE], [0], [0.0]))
        ctx.solve(tol=0.0, max_iters=K)
        g = ctx.get(0)
        tr = ctx.get_trace(0)
    assert g["status"] == P.STATUS_ITERATION_LIMIT
    assert_trajectory_match(g, tr, ores, what=f"K={K}")


def test_cfg1_converged(P):
    inst = make_cfg1()
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    ores = oracle_run(lp, eta, 1e-8, 100000)
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(deltas([BASE], [0], [0.0]))
        ctx.solve(tol=1e-8, max_iters=100000)
        g = ctx.get(0)
        tr = ctx.get_trace(0)
    assert g["status"] == P.STATUS_OPTIMAL
    assert_trajectory_match(g, tr, ores, rtol=1e-8, what="cfg1 1e-8")
    assert abs(g["obj"] - ores.obj) <= 1e-9 * (1 + abs(ores.obj))
    assert abs(g["kkt"][3] - ores.kkt.rel) <= 1e-6 * ores.kkt.rel + 1e-15


def test_step_size_matches_power_iteration(P):
    inst = make_cfg2(m=300, n=700)
    lp = O.from_instance(inst)
    with make_ctx(inst) as ctx:
        eta, na = ctx.step_size
    ref = np.linalg.norm(lp.A.toarray(), 2)
    assert math.isclose(na, ref, rel_tol=1e-9)
    assert math.isclose(eta, 0.998 / ref, rel_tol=1e-9)


# ---------------------------------------------------------------------------
# the strong-branching batch (B = 64, FP64, warm start) -- the benchmark workload
# ---------------------------------------------------------------------------

def _cfg2_ctx(P, inst, eta, base, D, **kw):
    ctx = make_ctx(inst, eta, **kw)
    ctx.set_batch(D, x_warm=base.x, y_warm=base.y, w_warm=np.full(len(D), base.w))
    return ctx


# K = C + 2 (18, 34, 66): the limit falls on the first iteration after a full
# evaluation, so the evaluation of fresh cycles there must run although no LP
# starts a cycle
@pytest.mark.parametrize("C", [64, 32, 16])
@pytest.mark.parametrize("K", [1, 18, 34, 65, 66, 200])
def test_cfg2_batch_fixed_iterations(P, K, C):
    inst, lp, eta, base, D = cfg2_setup()
    with _cfg2_ctx(P, inst, eta, base, D, eval_every=C) as ctx:
        ctx.solve(tol=0.0, max_iters=K)
        res = [(ctx.get(j), ctx.get_trace(j)) for j in range(len(D))]
    worst = 0.0
    for j, d in enumerate(D):
        ores = oracle_run(lp_for(lp, d), eta, 0.0, K, base.x, base.y, base.w, eval_every=C)
        worst = max(worst, assert_trajectory_match(*res[j], ores, what=f"LP {j} K={K} C={C}"))
    print(f"cfg2 K={K} C={C}: worst rel err {worst:.2e}")


# C = 32 is the evaluation interval the 2000 x 5000 strong-branching batch runs
# with, 24 the 200k x 500k line's, 16 serving's and 8 the line's one-at-a-time leg's
@pytest.mark.parametrize("C", [64, 32, 24, 16, 8])
def test_cfg2_batch_converged(P, C):
    inst, lp, eta, base, D = cfg2_setup()
    with _cfg2_ctx(P, inst, eta, base, D, eval_every=C) as ctx:
        ctx.solve(tol=1e-4, max_iters=100000)
        out = ctx.get_batch()
        traces = [ctx.get_trace(j) for j in range(len(D))]
    opt = out["status"] == P.STATUS_OPTIMAL
    assert opt.sum() >= len(D) - 2
    assert np.all(out["kkt"][opt, 3] <= 1e-4)
    same_traj = 0
    for j, d in enumerate(D):
        ores = oracle_run(lp_for(lp, d), eta, 1e-4, 100000, base.x, base.y, base.w,
                          eval_every=C)
        assert out["status"][j] == ores.status, (j, out["status"][j], ores.status)
        if ores.status == O.OPTIMAL:
            assert abs(out["obj"][j] - ores.obj) <= 4e-4 * (1 + abs(ores.obj)), j
        if out["iters"][j] == ores.iters and traces[j]["restart_log"] == ores.restarts:
            same_traj += 1
            assert rel_err(out["X"][j], ores.x) <= ITER_RTOL
            assert elem_err(out["X"][j], ores.x) <= ITER_RTOL
    # identical trajectories are expected for every LP (no restart test near a tie)
    assert same_traj == len(D)


@pytest.mark.parametrize("C, S", [(32, 8), (24, 8), (24, 4)])
def test_cfg2_batch_converged_with_stop_tests(P, C, S):
    """Stopping tests every S iterations between the full evaluations: the
    batch (restart tests, compaction and moves now also at the stopping tests)
    follows the oracle run with the same schedule, LP by LP: statuses,
    iteration counts, restart logs and iterates; and no LP stops later than
    without the tests."""
    inst, lp, eta, base, D = cfg2_setup()
    outs = {}
    for stop in (0, S):
        with _cfg2_ctx(P, inst, eta, base, D, eval_every=C, stop_every=stop) as ctx:
            ctx.solve(tol=1e-4, max_iters=100000)
            out = ctx.get_batch()
            out["traces"] = [ctx.get_trace(j) for j in range(len(D))]
            outs[stop] = out
    out = outs[S]
    assert np.all(out["iters"] <= outs[0]["iters"])
    assert np.any(out["iters"] < outs[0]["iters"])
    for j, d in enumerate(D):
        ores = oracle_run(lp_for(lp, d), eta, 1e-4, 100000, base.x, base.y, base.w,
                          eval_every=C, stop_every=S)
        g = {"status": out["status"][j], "iters": out["iters"][j], "x": out["X"][j],
             "y": out["Y"][j], "kkt": out["kkt"][j], "obj": out["obj"][j]}
        assert_trajectory_match(g, out["traces"][j], ores, what=(C, S, j))


def test_batched_equals_independent(P):
    """Each LP's result does not depend on the batch around it: bitwise equal
    alone (B = 1), in a small batch, and in the full batch."""
    inst, lp, eta, base, D = cfg2_setup()

    def run(idx):
        with make_ctx(inst, eta) as ctx:
            sub = D[idx]
            ctx.set_batch(sub, x_warm=base.x, y_warm=base.y, w_warm=np.full(len(sub), base.w))
            ctx.solve(tol=1e-4, max_iters=100000)
            return ctx.get_batch()

    full = run(np.arange(len(D)))
    small = run(np.array([5, 40, 17]))
    for pos, j in enumerate([5, 40, 17]):
        alone = run(np.array([j]))
        for other in (small, ):
            np.testing.assert_array_equal(other["X"][pos], full["X"][j])
            np.testing.assert_array_equal(other["Y"][pos], full["Y"][j])
            assert other["iters"][pos] == full["iters"][j]
        np.testing.assert_array_equal(alone["X"][0], full["X"][j])
        np.testing.assert_array_equal(alone["Y"][0], full["Y"][j])
        assert alone["iters"][0] == full["iters"][j]


def test_repeat_runs_bitwise_identical(P):
    inst, lp, eta, base, D = cfg2_setup()
    outs = []
    for _ in range(2):
        with _cfg2_ctx(P, inst, eta, base, D) as ctx:
            ctx.solve(tol=1e-4, max_iters=100000)
            outs.append(ctx.get_batch())
    np.testing.assert_array_equal(outs[0]["X"], outs[1]["X"])
    np.testing.assert_array_equal(outs[0]["Y"], outs[1]["Y"])


@pytest.mark.parametrize("graphs", [0, 1])
def test_graph_replay_equals_eager(P, graphs):
    inst, lp, eta, base, D = cfg2_setup()
    ref = None
    with _cfg2_ctx(P, inst, eta, base, D, use_graphs=graphs) as ctx:
        ctx.solve(tol=1e-4, max_iters=100000)
        out = ctx.get_batch()
    with _cfg2_ctx(P, inst, eta, base, D, use_graphs=1 - graphs) as ctx:
        ctx.solve(tol=1e-4, max_iters=100000)
        ref = ctx.get_batch()
    np.testing.assert_array_equal(out["X"], ref["X"])
    np.testing.assert_array_equal(out["iters"], ref["iters"])


# ---------------------------------------------------------------------------
# batch shapes: several column tiles, ragged tails, tile overrides
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("B", [1, 3, 63, 65, 130, 257])
def test_ragged_batch_sizes(P, B):
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    rng = np.random.default_rng(B)
    kinds = rng.choice([BASE, SET_LO, SET_HI, OBJ_UNIT], size=B)
    vars_ = rng.integers(0, lp.n, size=B)
    vals = np.where(kinds == SET_LO, rng.uniform(0, 10, B).round(),
                    np.where(kinds == SET_HI, rng.uniform(0, 10, B).round(),
                             rng.choice([-1.0, 1.0], B)))
    D = deltas(kinds, vars_, vals)
    K = 130
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=0.0, max_iters=K)
        picks = sorted({0, B // 2, B - 1})
        res = {j: (ctx.get(j), ctx.get_trace(j)) for j in picks}
    for j in picks:
        ores = oracle_run(lp_for(lp, D[j]), eta, 0.0, K)
        assert_trajectory_match(*res[j], ores, what=f"B={B} LP {j}")


@pytest.mark.parametrize("lanes, vec", [(1, 1), (4, 2), (16, 4), (64, 1), (32, 2)])
def test_tile_overrides_agree(P, lanes, vec):
    """Every tile shape sums each row in the same order: results are bitwise equal."""
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(lp.n, 20, seed=3))
    outs = []
    for tl, tv in [(0, 0), (lanes, vec)]:
        with make_ctx(inst, eta, tile_lanes=tl, tile_vec=tv) as ctx:
            ctx.set_batch(D)
            ctx.solve(tol=1e-4, max_iters=20000)
            outs.append(ctx.get_batch())
    np.testing.assert_array_equal(outs[0]["X"], outs[1]["X"])
    np.testing.assert_array_equal(outs[0]["iters"], outs[1]["iters"])


# ---------------------------------------------------------------------------
# statuses and failure isolation
# ---------------------------------------------------------------------------

def test_statuses_and_isolation(P):
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = deltas([SET_LO, SET_LO, SET_HI, SET_LO, OBJ_UNIT, BASE],
               [3, 4, 5, 6, 7, 0],
               [11.0, np.nan, -1.0, np.inf, 1.0, 0.0])
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=1e-4, max_iters=20000)
        out = ctx.get_batch()
    assert list(out["status"]) == [P.STATUS_INFEASIBLE_BOUNDS, P.STATUS_INVALID_INPUT,
                                   P.STATUS_INFEASIBLE_BOUNDS, P.STATUS_INVALID_INPUT,
                                   P.STATUS_OPTIMAL, P.STATUS_OPTIMAL]
    assert out["iters"][0] == 0
    # the running LPs are unaffected by their failing neighbours
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D[4:])
        ctx.solve(tol=1e-4, max_iters=20000)
        ref = ctx.get_batch()
    np.testing.assert_array_equal(out["X"][4:], ref["X"])
    # bad arguments fail the call
    with make_ctx(inst, eta) as ctx:
        with pytest.raises(P.PdlpbError) as e:
            ctx.set_batch(deltas([SET_LO], [lp.n], [1.0]))
        assert e.value.code == P.EINVAL
        with pytest.raises(P.PdlpbError) as e:
            ctx.set_batch(deltas([9], [0], [1.0]))
        assert e.value.code == P.EINVAL
        with pytest.raises(P.PdlpbError) as e:
            ctx.solve()
        assert e.value.code == P.ESTATE
        ctx.set_batch(deltas([BASE], [0], [0.0]))
        with pytest.raises(P.PdlpbError) as e:
            ctx.get(0)
        assert e.value.code == P.ESTATE
        ctx.solve(tol=0.0, max_iters=7)
        g = ctx.get(0)
        assert g["status"] == P.STATUS_ITERATION_LIMIT and g["iters"] == 7
        with pytest.raises(P.PdlpbError) as e:
            ctx.solve()
        assert e.value.code == P.ESTATE


def test_nan_reaches_numerical_error(P):
    """An LP whose iterates become NaN stops with NUMERICAL_ERROR at its next
    evaluation, the reference solver agrees, and its neighbours finish."""
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    y_bad = np.zeros((2, lp.m))
    y_bad[0, 7] = np.nan
    x0 = np.zeros((2, lp.n))
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(deltas([BASE, BASE], [0, 0], [0.0, 0.0]), x_warm=x0, y_warm=y_bad,
                      warm_mode=P.WARM_PER_LP)
        ctx.solve(tol=1e-4, max_iters=20000)
        out = ctx.get_batch()
    ores = O.solve(lp, O.Options(step_size=eta), x_init=x0[0], y_init=y_bad[0])
    assert ores.status == O.NUMERICAL_ERROR
    assert out["status"][0] == P.STATUS_NUMERICAL_ERROR and out["iters"][0] == ores.iters
    assert out["status"][1] == P.STATUS_OPTIMAL


# ---------------------------------------------------------------------------
# bound tightening, mixed precision, batch-average restarts
# ---------------------------------------------------------------------------

def test_obbt_batch_fixed_iterations_fp64(P):
    inst = make_cfg3(m=2000, n=5000)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(lp.n, 8, seed=11))
    K = 300
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=0.0, max_iters=K)
        res = [(ctx.get(j), ctx.get_trace(j)) for j in range(len(D))]
    for j, d in enumerate(D):
        ores = oracle_run(lp_for(lp, d), eta, 0.0, K)
        assert_trajectory_match(*res[j], ores, what=f"OBBT LP {j}")


def test_mixed32_error_statement(P):
    """FP32 iterates and products with FP64 sums: each LP reaches 1e-4 relative
    KKT, its objective matches the FP64 run within the 1e-4 bracket, and the
    FP32 point re-measured in FP64 by the reference KKT stays near 1e-4."""
    inst = make_cfg3(m=2000, n=5000)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(lp.n, 16, seed=12))
    outs = {}
    for prec in (P.FP64, P.MIXED32):
        with make_ctx(inst, eta, precision=prec) as ctx:
            ctx.set_batch(D)
            ctx.solve(tol=1e-4, max_iters=50000)
            outs[prec] = ctx.get_batch()
    a, b = outs[P.FP64], outs[P.MIXED32]
    assert np.all(a["status"] == P.STATUS_OPTIMAL) and np.all(b["status"] == P.STATUS_OPTIMAL)
    err = np.abs(b["obj"] - a["obj"]) / (1 + np.abs(a["obj"]))
    print(f"MIXED32 vs FP64 objective: max {err.max():.2e} median {np.median(err):.2e}")
    assert err.max() <= 1e-3
    for j in range(0, len(D), 4):
        k = O.kkt(lp_for(lp, D[j]), b["X"][j], b["Y"][j])
        assert k.rel <= 2e-3, (j, k)


@pytest.mark.parametrize("C", [64, 32])
def test_batch_avg_matches_oracle(P, C):
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(lp.n, 4, seed=13))
    lps = [lp_for(lp, d) for d in D]
    for tol, K in [(0.0, 400), (1e-5, 100000)]:
        ores = O.solve_batch_avg(lps, O.Options(tol=tol, max_iters=K, step_size=eta,
                                                eval_every=C))
        with make_ctx(inst, eta, restart_scope=P.RESTART_BATCH_AVG, eval_every=C) as ctx:
            ctx.set_batch(D)
            ctx.solve(tol=tol, max_iters=K)
            for j in range(len(D)):
                assert_trajectory_match(ctx.get(j), ctx.get_trace(j), ores[j],
                                        rtol=1e-8, what=f"avg tol={tol} LP {j}")


@pytest.mark.parametrize("C", [64, 32])
def test_infeasible_and_unbounded_lps_detected(P, C):
    """Section 4 infeasibility tests on the GPU: an infeasible box-constrained
    LP and an unbounded LP, each in a batch with a feasible neighbour; the
    statuses and the iteration at which each LP stops equal the oracle's."""
    import scipy.sparse as sp
    from workloads.generators import LPInstance
    # rows: x0 + x1 = 5 (E), x0 - x1 <= 3 (L); box [0, 1]^2 (infeasible) / [0, 4]^2 (feasible)
    A = sp.csr_matrix(np.array([[1.0, 1.0], [1.0, -1.0]]))
    def inst(hi):
        return LPInstance(m=2, n=2, row_ptr=A.indptr.astype(np.int64), col_idx=A.indices,
                          val=A.data, c=np.array([1.0, -1.0]), b=np.array([5.0, 3.0]),
                          sense=np.frombuffer(b"EL", dtype=np.uint8), l=np.zeros(2),
                          u=np.full(2, hi), x0=np.zeros(2))
    base_lp = O.from_instance(inst(4.0))
    eta = O.step_size(base_lp.A)
    D = deltas([SET_HI, BASE], [0, 0], [0.5, 0.0])                 # x0 <= 0.5 -> x1 >= 4.5 > 4
    with make_ctx(inst(4.0), eta, eval_every=C) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=1e-8, max_iters=200000)
        out = ctx.get_batch()
    assert list(out["status"]) == [P.STATUS_PRIMAL_INFEASIBLE, P.STATUS_OPTIMAL]
    for j, d in enumerate(D):
        r = oracle_run(lp_for(base_lp, d), eta, 1e-8, 200000, eval_every=C)
        assert (out["status"][j], out["iters"][j]) == (r.status, r.iters), (j, C)
    # unbounded: min -x0 s.t. x0 - x1 = 0, x >= 0 with no upper bounds
    B1 = sp.csr_matrix(np.array([[1.0, -1.0]]))
    unb = LPInstance(m=1, n=2, row_ptr=B1.indptr.astype(np.int64), col_idx=B1.indices, val=B1.data,
                     c=np.array([-1.0, 0.0]), b=np.zeros(1), sense=np.frombuffer(b"E", np.uint8),
                     l=np.zeros(2), u=np.full(2, np.inf), x0=np.zeros(2))
    unb_lp = O.from_instance(unb)
    eta = O.step_size(unb_lp.A)
    D = deltas([BASE, OBJ_UNIT], [0, 1], [0.0, 1.0])                # min -x0 (unbounded), min x1
    with make_ctx(unb, eta, eval_every=C) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=1e-8, max_iters=200000)
        out = ctx.get_batch()
    assert list(out["status"]) == [P.STATUS_DUAL_INFEASIBLE, P.STATUS_OPTIMAL]
    for j, d in enumerate(D):
        r = oracle_run(lp_for(unb_lp, d), eta, 1e-8, 200000, eval_every=C)
        assert (out["status"][j], out["iters"][j]) == (r.status, r.iters), (j, C)


def test_tiny_lps_reach_exact_optimum(P):
    """Brute-force optimum of tiny LPs through the whole GPU path."""
    from tests.lp_exact import vertex_enum
    for seed in range(4):
        inst = make_tiny(seed, m=3, n=5, senses="ELG", box=(0.0, 4.0))
        lp = O.from_instance(inst)
        best, _ = vertex_enum(lp.A.toarray(), lp.l, lp.u, lp.xl, lp.xu, lp.c)
        with make_ctx(inst) as ctx:
            ctx.set_batch(deltas([BASE], [0], [0.0]))
            ctx.solve(tol=1e-9, max_iters=400000)
            g = ctx.get(0)
        assert g["status"] == P.STATUS_OPTIMAL
        assert abs(g["obj"] - best) <= 1e-7 * (1 + abs(best)), seed


def test_autotune_leaves_results_unchanged(P):
    """The tile-shape timing runs inside the first block of iterations of a
    large batch; every shape gives the same bits, so results match a run with
    the fixed heuristic shape."""
    inst = make_cfg3(m=20000, n=50000)
    D = obbt_deltas(choose_vars(inst.n, 48, seed=21))
    outs = []
    for tune in (0, 1):
        with make_ctx(inst, 0.05, autotune=tune) as ctx:
            ctx.set_batch(D)
            ctx.solve(tol=0.0, max_iters=200)
            outs.append(ctx.get_batch())
    np.testing.assert_array_equal(outs[0]["X"], outs[1]["X"])
    np.testing.assert_array_equal(outs[0]["Y"], outs[1]["Y"])
    np.testing.assert_array_equal(outs[0]["iters"], outs[1]["iters"])


def test_caller_stream_and_device_buffers(P):
    """A context on a stream the caller owns (a torch stream of default
    priority), inputs and outputs in device memory: the batch gives the same
    bits as on the context's own stream, and a torch operation queued on the
    caller's stream right after get_batch sees the finished results."""
    import torch
    inst, lp, eta, base, D = cfg2_setup()
    with make_ctx(inst, eta, eval_every=32) as ctx:
        ctx.set_batch(D, x_warm=base.x, y_warm=base.y, w_warm=np.full(len(D), base.w))
        ctx.solve(tol=1e-4, max_iters=100000)
        ref = ctx.get_batch()
    s = torch.cuda.Stream()
    dev = torch.device("cuda:0")
    with torch.cuda.stream(s):
        with make_ctx(inst, eta, eval_every=32, stream=s.cuda_stream) as ctx:
            dD = torch.from_numpy(D.view(np.uint8).copy()).to(dev)
            dx = torch.from_numpy(base.x).to(dev)
            dy = torch.from_numpy(base.y).to(dev)
            dw = torch.full((len(D),), base.w, dtype=torch.float64, device=dev)
            ctx.set_batch(dD, x_warm=dx, y_warm=dy, w_warm=dw, mem=P.MEM_DEVICE)
            ctx.solve(tol=1e-4, max_iters=100000)
            X = torch.empty((len(D), inst.n), dtype=torch.float64, device=dev)
            Y = torch.empty((len(D), inst.m), dtype=torch.float64, device=dev)
            out = ctx.get_batch(X=X, Y=Y, mem=P.MEM_DEVICE)
            row_sums = X.sum(dim=1)               # queued on the caller's stream
    s.synchronize()
    np.testing.assert_array_equal(out["status"], ref["status"])
    np.testing.assert_array_equal(out["iters"], ref["iters"])
    np.testing.assert_array_equal(X.cpu().numpy(), ref["X"])
    np.testing.assert_array_equal(Y.cpu().numpy(), ref["Y"])
    np.testing.assert_allclose(row_sums.cpu().numpy(), ref["X"].sum(axis=1), rtol=1e-12)


def test_binding_checks_arrays_it_passes_by_address(P):
    """The library reads and writes device arrays through bare addresses, so
    the binding refuses what would send it past an array's end or into the
    wrong type: host arrays given as device memory, FP32 or strided tensors,
    too few entries for the warm-start mode, and result tensors too small for
    the batch.  A refused call changes nothing; the right arrays then work."""
    import torch
    inst, lp, eta, base, D = cfg2_setup()
    dev = torch.device("cuda:0")
    B = 8
    dD = torch.from_numpy(D[:B].view(np.uint8).copy()).to(dev)
    dx = torch.from_numpy(base.x).to(dev)
    dy = torch.from_numpy(base.y).to(dev)
    dw = torch.full((B,), base.w, dtype=torch.float64, device=dev)
    M = P.MEM_DEVICE
    with make_ctx(inst, eta, eval_every=32) as ctx:
        bad = [
            (TypeError, dict(deltas=D[:B])),
            (ValueError, dict(deltas=dD[:40])),
            (TypeError, dict(x_warm=dx.float())),
            (TypeError, dict(x_warm=torch.stack([dx, dx], 1)[:, 0])),
            (ValueError, dict(x_warm=dx, warm_mode=P.WARM_PER_LP)),
            (ValueError, dict(y_warm=dy[:-1], warm_mode=P.WARM_SHARED)),
            (ValueError, dict(w_warm=dw[:B - 1])),
        ]
        for err, kw in bad:
            args = dict(deltas=dD, x_warm=dx, y_warm=dy, w_warm=dw, mem=M)
            args.update(kw)
            with pytest.raises(err):
                ctx.set_batch(args.pop("deltas"), **args)
        with pytest.raises(ValueError):
            ctx.set_batch(D[:B], x_warm=base.x[:-1], y_warm=base.y)
        ctx.set_batch(dD, x_warm=dx, y_warm=dy, w_warm=dw, mem=M)
        ctx.solve(tol=1e-4, max_iters=100000)
        X = torch.empty((B, inst.n), dtype=torch.float64, device=dev)
        Y = torch.empty((B, inst.m), dtype=torch.float64, device=dev)
        with pytest.raises(ValueError):
            ctx.get_batch(X=X[:B - 1], Y=Y, mem=M)
        with pytest.raises(TypeError):
            ctx.get_batch(X=X.float(), Y=Y, mem=M)
        out = ctx.get_batch(X=X, Y=Y, mem=M)
        ref = ctx.get_batch()
    assert np.array_equal(X.cpu().numpy(), ref["X"]) and np.array_equal(Y.cpu().numpy(), ref["Y"])
    assert np.array_equal(out["status"], ref["status"])


@pytest.mark.parametrize("K", [1, 66, 200])
def test_per_lp_warm_starts(P, K):
    """Each LP starts from its own primal point (partly outside the box, which
    the start projects onto), its own dual point and its own primal weight; the
    iterates, statuses and restart iterations after K iterations equal the
    oracle's started the same way."""
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    rng = np.random.default_rng(11)
    B = 7
    D = obbt_deltas(choose_vars(inst.n, 3, seed=5))[:B - 1]
    D = np.concatenate([deltas([BASE], [0], [0.0]), D])
    X0 = rng.uniform(-2.0, 12.0, size=(B, inst.n))          # box [0, 10]
    Y0 = rng.normal(size=(B, inst.m))
    W0 = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=B))
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D, x_warm=X0.ravel(), y_warm=Y0.ravel(), w_warm=W0,
                      warm_mode=P.WARM_PER_LP)
        ctx.solve(tol=0.0, max_iters=K)
        res = [(ctx.get(j), ctx.get_trace(j)) for j in range(B)]
    for j, d in enumerate(D):
        ores = oracle_run(lp_for(lp, d), eta, 0.0, K, X0[j], Y0[j], W0[j])
        assert_trajectory_match(*res[j], ores, what=f"LP {j} K={K}")


def test_graphs_are_reused_across_batches(P):
    """Blocks of C iterations captured for one batch are replayed for later
    batches of the same launch shape instead of being captured again, and the
    replays give the bits of the first solve; B = 1 batches solved one after
    another share one set of graphs too."""
    inst, lp, eta, base, D = cfg2_setup()
    with _cfg2_ctx(P, inst, eta, base, D, eval_every=32) as ctx:
        ctx.solve(tol=1e-4, max_iters=100000)
        first = ctx.get_batch()
        n1 = ctx.graph_captures
        assert n1 >= 1
        for _ in range(3):
            ctx.set_batch(D, x_warm=base.x, y_warm=base.y, w_warm=np.full(len(D), base.w))
            ctx.solve(tol=1e-4, max_iters=100000)
            again = ctx.get_batch()
            np.testing.assert_array_equal(again["iters"], first["iters"])
            np.testing.assert_array_equal(again["X"], first["X"])
            np.testing.assert_array_equal(again["Y"], first["Y"])
        assert ctx.graph_captures == n1
        ones = []
        for j in range(6):
            ctx.set_batch(D[j:j + 1], x_warm=base.x, y_warm=base.y, w_warm=np.full(1, base.w))
            ctx.solve(tol=1e-4, max_iters=100000)
            ones.append(ctx.get_batch())
            if j == 0:
                n2 = ctx.graph_captures
        assert ctx.graph_captures == n2
        for j, o in enumerate(ones):
            assert o["iters"][0] == first["iters"][j]
            np.testing.assert_array_equal(o["X"][0], first["X"][j])
