"""Precision statement of the mixed mode at the full bound-tightening size:
A 20000 x 50000 with 8 U[-1,1] nonzeros per column, E/L/G rows, box [0,5];
256 LPs minimising and maximising 128 variables, cold start, tol 1e-4.  FP32
iterates and products with FP64 sums against the FP64 run of the same batch,
and every FP32 point re-measured by the oracle's FP64 KKT, both against A
itself and against A rounded to FP32 (the matrix the FP32 run multiplies by),
which separates the data rounding from the iteration's own error.  At a
smaller size, the mixed-mode iterates after a fixed number of iterations
against the FP64 oracle, within the growth of FP32 rounding."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from tests.gpu_common import make_ctx, lp_for
from workloads import make_cfg3, obbt_deltas, choose_vars, seed_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


def test_mixed32_precision_statement_full_size(P):
    inst = make_cfg3()
    lp = O.from_instance(inst)
    D = obbt_deltas(choose_vars(inst.n, 128, seed_for(3, 0)))
    outs = {}
    for prec in (P.FP64, P.MIXED32):
        with make_ctx(inst, precision=prec) as ctx:
            ctx.set_batch(D)
            ctx.solve(tol=1e-4, max_iters=100000)
            outs[prec] = ctx.get_batch()
    a, b = outs[P.FP64], outs[P.MIXED32]
    both = (a["status"] == P.STATUS_OPTIMAL) & (b["status"] == P.STATUS_OPTIMAL)
    assert both.mean() >= 0.95, np.bincount(b["status"])
    err = np.abs(b["obj"] - a["obj"]) / (1 + np.abs(a["obj"]))
    A32 = sp.csr_matrix((inst.val.astype(np.float32).astype(np.float64), inst.col_idx,
                         inst.row_ptr), shape=(inst.m, inst.n))
    rel, rel32, dev = [], [], []
    for j in np.nonzero(both)[0][::8]:
        lpj = lp_for(lp, D[j])
        rel.append(O.kkt(lpj, b["X"][j], b["Y"][j]).rel)
        lpj32 = O.LP(A=A32, c=lpj.c, l=lpj.l, u=lpj.u, xl=lpj.xl, xu=lpj.xu, b=lpj.b)
        rel32.append(O.kkt(lpj32, b["X"][j], b["Y"][j]).rel)
        dev.append(float(b["kkt"][j, 3]))
    gap_dev = max(abs(r - d) for r, d in zip(rel32, dev))
    print(f"MIXED32 vs FP64 objective over {both.sum()} LPs: max {err[both].max():.2e} "
          f"median {np.median(err[both]):.2e}; oracle KKT of FP32 points: max {max(rel):.2e} "
          f"median {np.median(rel):.2e} (vs FP32-rounded A: max {max(rel32):.2e}; "
          f"|oracle - device| max {gap_dev:.2e})")
    assert err[both].max() <= 1e-3
    # Against the FP32-rounded A, the matrix the FP32 run multiplies by, the oracle
    # measures what the device's FP64 sums measured: the same number up to
    # summation order, and within the stopping tolerance.
    assert gap_dev <= 1e-9
    assert max(rel32) <= 1e-4 * (1 + 1e-6)
    # Against A itself the measure also carries the rounding of A's entries
    # (relative 6e-8), amplified by the norms of the iterates; on this batch the
    # points still meet the tolerance against A (measured max 3.5e-5), so the
    # FP32 LPs counted as solved are solved for the LP as given.
    assert max(rel) <= 1e-4


@pytest.mark.parametrize("K", [1, 2, 8, 32, 64])
def test_mixed32_fixed_iterations_within_rounding_growth(P, K):
    """The mixed mode runs the oracle's iteration: after K iterations its
    iterates differ from the FP64 oracle's by at most 4 (K + 1) u relative,
    u = 2^-24.  Each iteration rounds to FP32 at most four times what it feeds
    forward (the primal and dual points of T, the Halpern combination, and A
    itself), and the reflected step is nonexpansive, so these errors add up
    without growing.  K <= 64 keeps every decision (stopping, infeasibility,
    restart) out of the run: with tol = 0 the only full evaluation is at
    t = 0, so statuses, counts and restart logs must also agree exactly."""
    from tests.gpu_common import oracle_run, rel_err
    inst = make_cfg3(m=2000, n=5000)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(lp.n, 4, seed=12))
    with make_ctx(inst, eta, precision=P.MIXED32) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=0.0, max_iters=K)
        res = [(ctx.get(j), ctx.get_trace(j)) for j in range(len(D))]
    bound = 4 * (K + 1) * 2.0 ** -24
    for j, d in enumerate(D):
        o = oracle_run(lp_for(lp, d), eta, 0.0, K)
        g, tr = res[j]
        assert (g["status"], g["iters"], tr["restart_log"]) == (o.status, o.iters, o.restarts[:64])
        errs = (rel_err(g["x"], o.x), rel_err(g["y"], o.y), rel_err(tr["x_iter"], o.x_iter),
                rel_err(tr["y_iter"], o.y_iter))
        assert max(errs) <= bound, (j, K, errs, bound)


def test_mixed32_bound_tightening_batch_sampled_fixed_iterations(P):
    """The bound-tightening batch as the benchmark runs it (A 20000 x 50000,
    256 LPs, FP32 iterates, default options with the tile autotuner) after 64
    iterations: every LP is still running with 64 iterations, and sampled LPs
    recomputed one at a time by the FP64 oracle agree within 4 (K + 1) u, the
    bound of the fixed-iteration test above."""
    from tests.gpu_common import oracle_run, rel_err
    inst = make_cfg3()
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(inst.n, 128, seed_for(3, 0)))
    K = 64
    sample = [0, 127, 128, 255]
    with make_ctx(inst, eta, precision=P.MIXED32) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=0.0, max_iters=K)
        st = ctx.get_batch(want_x=False, want_y=False)
        res = {j: (ctx.get(j), ctx.get_trace(j)) for j in sample}
    assert np.all(st["iters"] == K) and np.all(st["status"] == P.STATUS_ITERATION_LIMIT)
    bound = 4 * (K + 1) * 2.0 ** -24
    for j in sample:
        o = oracle_run(lp_for(lp, D[j]), eta, 0.0, K)
        g, tr = res[j]
        errs = (rel_err(g["x"], o.x), rel_err(g["y"], o.y), rel_err(tr["x_iter"], o.x_iter),
                rel_err(tr["y_iter"], o.y_iter))
        print(f"LP {j}: {max(errs):.2e} (bound {bound:.2e})")
        assert max(errs) <= bound, (j, errs, bound)
