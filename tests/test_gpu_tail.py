"""The persistent tail through the C ABI: once at most tail_cols LPs of a batch
still run, one workgroup per LP finishes them in one launch.  Its results
equal the batched kernels' bit for bit (iterates, statuses, iteration counts,
KKT measures, restart logs, primal weights) on converged batches, at fixed
iteration counts, with iteration limits inside a block of C iterations, in
FP64 and with FP32 iterates; and they match the oracle's trajectories."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import cfg2_setup, make_ctx, lp_for, oracle_run, assert_trajectory_match
from workloads import make_cfg2, choose_fractional, fsb_deltas, obbt_deltas, choose_vars, seed_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


def _run(P, inst, eta, D, tol, K, tail, warm=None, **kw):
    with make_ctx(inst, eta, tail_cols=tail, **kw) as ctx:
        if warm is None:
            ctx.set_batch(D)
        else:
            ctx.set_batch(D, x_warm=warm.x, y_warm=warm.y, w_warm=np.full(len(D), warm.w))
        ctx.set_kernel_timing(True)
        ctx.solve(tol=tol, max_iters=K)
        cnt, _ = ctx.kernel_times()
        out = ctx.get_batch()
        out["dobj"] = ctx.dual_objective()
        out["traces"] = [ctx.get_trace(j) for j in range(len(D))]
        out["tail_launches"] = cnt[4]
    return out


def _same(a, b):
    for key in ("X", "Y", "status", "iters", "kkt", "obj", "dobj"):
        assert np.array_equal(a[key], b[key], equal_nan=True), key
    for ta, tb in zip(a["traces"], b["traces"]):
        assert np.array_equal(ta["x_iter"], tb["x_iter"])
        assert np.array_equal(ta["y_iter"], tb["y_iter"])
        assert ta["w"] == tb["w"] and ta["restart_log"] == tb["restart_log"]


@pytest.mark.parametrize("prec, stop", [("fp64", 0), ("fp32", 0), ("fp64", 8)])
def test_tail_equals_batched_kernels_converged(P, prec, stop):
    """The 2000 x 5000 strong-branching batch (64 LPs, warm start, one
    infeasible branch in the family): the last LPs finish in the tail; with
    stop = 8 both also run stopping tests between the full evaluations."""
    inst, lp, eta, base, D = cfg2_setup()
    precision = P.MIXED32 if prec == "fp32" else P.FP64
    a = _run(P, inst, eta, D, 1e-4, 100000, 8, warm=base, precision=precision, eval_every=32,
             stop_every=stop)
    b = _run(P, inst, eta, D, 1e-4, 100000, 0, warm=base, precision=precision, eval_every=32,
             stop_every=stop)
    assert a["tail_launches"] == 1 and b["tail_launches"] == 0
    _same(a, b)


@pytest.mark.parametrize("K", [1, 33, 150, 257])
def test_tail_equals_batched_kernels_fixed_iterations(P, K):
    """Iteration limits at, before and inside blocks of C = 64 iterations;
    a batch of five LPs runs in the tail right after its first evaluation."""
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(inst.n, 3, seed=K))[:5]
    a = _run(P, inst, eta, D, 0.0, K, 8)
    b = _run(P, inst, eta, D, 0.0, K, 0)
    assert b["tail_launches"] == 0
    _same(a, b)
    assert all(s == P.STATUS_ITERATION_LIMIT for s in a["status"])
    assert all(int(i) == K for i in a["iters"])


def test_tail_matches_oracle(P):
    """LPs iterated in the tail from their first block on follow the oracle's
    trajectories (statuses, iteration counts, restart logs, iterates within
    1e-9), converged and at a fixed iteration count."""
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    root = O.solve(lp, O.Options(tol=1e-7, step_size=eta))
    D = fsb_deltas(root.x, choose_fractional(root.x, 2, seed_for(2, 77)))
    for tol, K in ((1e-6, 20000), (0.0, 300)):
        with make_ctx(inst, eta, tail_cols=8) as ctx:
            ctx.set_batch(D, x_warm=root.x, y_warm=root.y, w_warm=np.full(len(D), root.w))
            ctx.set_kernel_timing(True)
            ctx.solve(tol=tol, max_iters=K)
            assert ctx.kernel_times()[0][4] == 1
            for j, d in enumerate(D):
                g = ctx.get(j)
                tr = ctx.get_trace(j)
                ref = oracle_run(lp_for(lp, d), eta, tol, K, root.x, root.y, root.w)
                assert_trajectory_match(g, tr, ref, what=(tol, j))
