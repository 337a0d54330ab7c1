"""Precision statement of the mixed mode at the full bound-tightening size:
A 20000 x 50000 with 8 U[-1,1] nonzeros per column, E/L/G rows, box [0,5];
256 LPs minimising and maximising 128 variables, cold start, tol 1e-4.  FP32
iterates and products with FP64 sums against the FP64 run of the same batch,
and every FP32 point re-measured by the oracle's FP64 KKT, both against A
itself and against A rounded to FP32 (the matrix the FP32 run multiplies by),
which separates the data rounding from the iteration's own error."""
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
    rel, rel32 = [], []
    for j in np.nonzero(both)[0][::8]:
        lpj = lp_for(lp, D[j])
        rel.append(O.kkt(lpj, b["X"][j], b["Y"][j]).rel)
        lpj32 = O.LP(A=A32, c=lpj.c, l=lpj.l, u=lpj.u, xl=lpj.xl, xu=lpj.xu, b=lpj.b)
        rel32.append(O.kkt(lpj32, b["X"][j], b["Y"][j]).rel)
    print(f"MIXED32 vs FP64 objective over {both.sum()} LPs: max {err[both].max():.2e} "
          f"median {np.median(err[both]):.2e}; oracle KKT of FP32 points: max {max(rel):.2e} "
          f"(vs FP32-rounded A: max {max(rel32):.2e})")
    assert err[both].max() <= 1e-3
    assert max(rel) <= 2e-3 and max(rel32) <= 2e-3
