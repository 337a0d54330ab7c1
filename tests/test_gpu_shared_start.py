"""The shared start through the C ABI: a batch whose running LPs all start from
one point with the same primal weight makes its first iteration and
evaluation once per base LP and per LP only where its change reaches, and
writes the dense blocks only for the LPs still running after t = 0.  Its
results equal the full-width path's bit for bit (iterates, Halpern iterates,
statuses, iteration counts, KKT measures, objectives, restart logs, primal
weights): bound changes and objective changes, both base LPs in one batch,
LPs settled at submission, budgets of one and two iterations, loose
tolerances that stop most LPs at t = 0, the batch-average restart scope,
stopping tests between evaluations, FP32 iterates, a scaled LP, evaluation
chains longer than 64 rows, and batches holding a change beyond the per-LP
kernels' reach, which take the full-width path."""
import numpy as np
import pytest

from tests.gpu_common import cfg2_setup, make_ctx
from workloads import (fsb_deltas, obbt_deltas, choose_vars, deltas, make_packing, make_facility,
                       BASE, SET_LO, SET_HI)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


def _run(inst, eta, D, tol, K, shared, warm=None, w=None, **kw):
    with make_ctx(inst, eta, shared_start=shared, **kw) as ctx:
        if warm is None:
            ctx.set_batch(D, w_warm=w)
        else:
            ctx.set_batch(D, x_warm=warm.x, y_warm=warm.y,
                          w_warm=np.full(len(D), warm.w) if w is None else w)
        ctx.set_kernel_timing(True)
        ctx.solve(tol=tol, max_iters=K)
        cnt, _ = ctx.kernel_times()
        out = ctx.get_batch()
        out["dobj"] = ctx.dual_objective()
        out["traces"] = [ctx.get_trace(j) for j in range(len(D))]
        out["launches"] = cnt
    return out


def _same(a, b):
    for key in ("X", "Y", "status", "iters", "kkt", "obj", "dobj"):
        assert np.array_equal(a[key], b[key], equal_nan=True), key
    for j, (ta, tb) in enumerate(zip(a["traces"], b["traces"])):
        assert np.array_equal(ta["x_iter"], tb["x_iter"], equal_nan=True), ("x_iter", j)
        assert np.array_equal(ta["y_iter"], tb["y_iter"], equal_nan=True), ("y_iter", j)
        assert ta["w"] == tb["w"] and ta["restart_log"] == tb["restart_log"], j


def _both(inst, eta, D, tol, K, **kw):
    a = _run(inst, eta, D, tol, K, 1, **kw)
    b = _run(inst, eta, D, tol, K, -1, **kw)
    # the shared start skips the full-width iteration at t = 0
    assert a["launches"][0] == b["launches"][0] - 1
    _same(a, b)
    return a


@pytest.mark.parametrize("prec, C, stop", [("fp64", 32, 0), ("fp32", 32, 0), ("fp64", 32, 8),
                                           ("fp64", 8, 0)])
def test_strong_branching_from_the_root(P, prec, C, stop):
    """64 bound changes on the 2000 x 5000 family, warm start from the root."""
    inst, lp, eta, base, D = cfg2_setup()
    precision = P.MIXED32 if prec == "fp32" else P.FP64
    for tol, K in ((1e-4, 100000), (1e-2, 100000), (0.0, 1), (0.0, 2), (0.0, 70)):
        _both(inst, eta, D, tol, K, warm=base, precision=precision, eval_every=C, stop_every=stop)


def test_loose_tolerance_stops_most_lps_at_the_first_evaluation(P):
    """At 1e-3 about half of the batch meets the tolerance at z~ = T(z^0) (the
    reference solver's KKT measures there run from 8e-5 to 3e-3), so the first
    compaction retires LPs on both sides of the new column count and moves
    running ones into the freed slots."""
    inst, lp, eta, base, D = cfg2_setup()
    out = _both(inst, eta, D, 1e-3, 100000, warm=base, eval_every=16)
    stopped_first = int(np.sum(out["iters"] == 1))
    assert len(D) // 4 < stopped_first < 3 * len(D) // 4


@pytest.mark.parametrize("warm", [False, True])
def test_objective_and_bound_changes_in_one_batch(P, warm):
    """Both base LPs: bound tightening (objective 0 but one entry) next to
    branching changes and the base LP itself, from zero and from the root."""
    inst, lp, eta, base, D = cfg2_setup()
    vars_ = choose_vars(inst.n, 10, seed=5)
    mix = np.concatenate([obbt_deltas(vars_), D[:24], deltas([BASE, BASE], [0, 0], [0.0, 0.0])])
    for tol, K in ((1e-4, 100000), (0.0, 1), (0.0, 40)):
        _both(inst, eta, mix, tol, K, warm=base if warm else None, eval_every=16)


def test_lps_settled_at_submission_and_batch_average_scope(P):
    inst, lp, eta, base, D = cfg2_setup()
    v = int(choose_vars(inst.n, 1, seed=9)[0])
    bad = deltas([SET_LO, SET_HI], [v, v], [float(inst.u[v]) + 1.0, float(inst.l[v]) - 1.0])
    mixed = np.concatenate([D[:20], bad, D[20:40]])
    out = _both(inst, eta, mixed, 1e-4, 100000, warm=base, eval_every=32)
    assert out["status"][20] == P.STATUS_INFEASIBLE_BOUNDS
    _both(inst, eta, D, 1e-4, 100000, warm=base, eval_every=32,
          restart_scope=P.RESTART_BATCH_AVG)


def test_scaled_lp(P):
    inst, lp, eta, base, D = cfg2_setup()
    _both(inst, None, D[:32], 1e-4, 100000, warm=base, eval_every=32, scaling=1)


def test_unequal_weights_take_the_full_width_path(P):
    """LPs with different primal weights do not share T(z^0): the option has
    nothing to do, the t = 0 iteration runs at full width either way."""
    inst, lp, eta, base, D = cfg2_setup()
    w = np.full(len(D), base.w)
    w[3] *= 1.5
    a = _run(inst, eta, D, 1e-4, 100000, 1, warm=base, w=w, eval_every=32)
    b = _run(inst, eta, D, 1e-4, 100000, -1, warm=base, w=w, eval_every=32)
    assert a["launches"][0] == b["launches"][0]
    _same(a, b)


def test_evaluation_chains_longer_than_a_wave(P):
    """600000 columns, 1000 packing rows, two nonzeros per column: the x
    chains of the evaluation hold 128 rows (two rounds of 64 lanes) and each
    changed variable reaches about 1200 columns."""
    inst = make_packing(rep=1, m=1000, n=600000, k=2)
    with make_ctx(inst, None, max_batch=1) as ctx:
        eta = ctx.step_size[0]
    vars_ = choose_vars(inst.n, 6, seed=3)
    D = np.concatenate([obbt_deltas(vars_), fsb_deltas(np.full(inst.n, 0.5), vars_)])
    for tol, K in ((0.0, 1), (0.0, 30)):
        _both(inst, eta, D, tol, K, eval_every=8)


@pytest.mark.parametrize("C", [32, 8])
def test_persistent_tail_after_the_shared_start(P, C):
    """The persistent tail takes the last LPs of converging batches
    (tail_cols = 8): it reads the blocks the shared start writes for the LPs
    still running, and its results equal the full-width path's bit for bit;
    at a fixed iteration count every LP runs to the cap together and neither
    path reaches the tail."""
    inst, lp, eta, base, D = cfg2_setup()
    for batch in (D, D[:10]):
        for tol, K in ((1e-4, 100000), (0.0, 40)):
            a = _run(inst, eta, batch, tol, K, 1, warm=base, eval_every=C, tail_cols=8)
            b = _run(inst, eta, batch, tol, K, -1, warm=base, eval_every=C, tail_cols=8)
            assert a["launches"][4] == b["launches"][4] == (1 if tol > 0 else 0)
            _same(a, b)


def _reach(inst):
    """Per variable v: the entries of column v of A, and the columns the rows
    through v reach (v counted once more), the coordinates a change of v moves
    in one LP's first evaluation."""
    import scipy.sparse as sp
    A = sp.csr_matrix((inst.val, inst.col_idx, inst.row_ptr), shape=(inst.m, inst.n))
    row_len = np.diff(inst.row_ptr)
    T = A.tocsc()
    ncol = np.diff(T.indptr)
    reach = np.array([1 + row_len[T.indices[T.indptr[v]:T.indptr[v + 1]]].sum()
                      for v in range(inst.n)])
    return ncol, reach


@pytest.mark.parametrize("F, C, k, cap", [(100, 1000, 10, "column"), (2, 9000, 1, "reach")])
def test_changes_beyond_the_per_lp_reach_take_the_full_width_path(P, F, C, k, cap):
    """The per-LP kernels of the shared start take a change of v when column v
    holds at most 64 entries and the rows through v reach at most 4096
    columns.  Facility location has both kinds beyond: a facility's column
    holds about C k / F entries, and with two facilities the capacity row
    through a customer's variable reaches thousands of columns.  A batch of
    changes within the reach takes the shared start; one change beyond it
    sends the whole batch down the full-width path; the bits are the same."""
    inst = make_facility(0, F=F, C=C, k=k)
    ncol, reach = _reach(inst)
    within = np.flatnonzero((ncol <= 64) & (reach <= 4096))
    beyond = np.flatnonzero(ncol > 64) if cap == "column" else \
        np.flatnonzero((ncol <= 64) & (reach > 4096))
    assert within.size >= 8 and beyond.size >= 1
    with make_ctx(inst, None, max_batch=1) as ctx:
        eta = ctx.step_size[0]
    rng = np.random.default_rng(F)
    good = obbt_deltas(np.sort(rng.choice(within, 4, replace=False)))
    mixed = np.concatenate([good[:3], obbt_deltas(rng.choice(beyond, 1)), good[3:]])
    for D, shared in ((good, True), (mixed, False)):
        for tol, K in ((0.0, 1), (0.0, 30), (1e-4, 2000)):
            a = _run(inst, eta, D, tol, K, 1, eval_every=8)
            b = _run(inst, eta, D, tol, K, -1, eval_every=8)
            assert a["launches"][0] == b["launches"][0] - (1 if shared else 0), (shared, K)
            _same(a, b)
