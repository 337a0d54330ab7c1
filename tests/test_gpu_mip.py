"""MIP-facing outputs through the C ABI against the oracle: the dual
objective, safe OBBT bounds with the improvement threshold (Section 5.2 and
the OBBT experiments of Section 6), strong-branching gains and scores
(Section 5.1), and the strict dual-feasibility tolerance."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle import mip as M
from tests.gpu_common import make_ctx, lp_for, oracle_run, cfg2_setup
from tests.lp_exact import highs
from workloads import (make_cfg2, make_packing, obbt_deltas, choose_vars, deltas, BASE,
                       SET_LO, SET_HI)

pytestmark = pytest.mark.gpu

RTOL = 1e-9


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


def _close(a, b, rtol=RTOL):
    if math.isinf(b) or math.isnan(b):
        return a == b or (math.isnan(a) and math.isnan(b))
    return abs(a - b) <= rtol * (1.0 + abs(b))


def test_obbt_bounds_match_oracle(P):
    """Packing rows (6 of the 8 upper bounds move): the GPU's dual objectives,
    tightened bounds and change count equal the oracle's, and every moved
    bound is safe against HiGHS's exact optimum."""
    inst = make_packing()
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(lp.n, 8, seed=21))
    tol, K = 1e-6, 40000
    with make_ctx(inst, eta, dual_tol=1e-8) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=tol, max_iters=K)
        got = ctx.get_batch(want_x=False, want_y=False)
        dobj = ctx.dual_objective()
        t_gpu = ctx.obbt_tighten(eps=M.OBBT_DUAL_TOL, min_improve=M.OBBT_MIN_IMPROVE)
    ores = [oracle_run(lp_for(lp, d), eta, tol, K, dual_tol=1e-8) for d in D]
    for j, r in enumerate(ores):
        assert got["status"][j] == r.status and got["iters"][j] == r.iters, j
        assert _close(dobj[j], r.kkt.dual_obj), (j, dobj[j], r.kkt.dual_obj)
    t = M.obbt_tighten(lp.xl, lp.xu, [int(d["var"]) for d in D], [float(d["value"]) for d in D],
                       ores)
    assert t.changed >= 4
    assert t_gpu["changed"] == t.changed and t_gpu["infeasible"] == t.infeasible
    for a, b in ((t_gpu["lo"], t.xl), (t_gpu["hi"], t.xu)):
        assert all(_close(float(u), float(v)) for u, v in zip(a, b))
    for d in D:
        v, s = int(d["var"]), float(d["value"])
        exact, _, _ = highs(lp_for(lp, d))          # min s * x_v
        if s > 0:
            assert t_gpu["lo"][v] <= exact + 1e-9
        else:
            assert t_gpu["hi"][v] >= -exact - 1e-9


def test_branch_scores_match_oracle(P):
    inst, lp, eta, base, D = cfg2_setup(m=200, n=500, p=6)
    tol, K = 1e-5, 20000
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D, x_warm=base.x, y_warm=base.y, w_warm=np.full(len(D), base.w))
        ctx.solve(tol=tol, max_iters=K)
        sc = ctx.branch_scores(base.obj)
    ores = [oracle_run(lp_for(lp, d), eta, tol, K, base.x, base.y, base.w) for d in D]
    gains = [M.branch_gain(r, base.obj) for r in ores]
    for j in range(len(D)):
        assert _close(sc["gain"][j], gains[j]), (j, sc["gain"][j], gains[j])
    p = len(D) // 2                 # LP i is the up branch of its variable, p + i the down
    for i in range(p):
        want = M.branch_score(gains[p + i], gains[i])
        assert _close(sc["score"][i], want) and _close(sc["score"][p + i], want), i


def test_branch_score_edge_cases(P):
    """An up branch that crosses the upper bound is infeasible (+inf gain and
    score); a variable with one branch only has no score; other kinds: NaN."""
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    parent = oracle_run(lp, eta, 1e-6, 40000)
    D = deltas([SET_LO, SET_HI, SET_LO, BASE], [3, 3, 7, 0], [11.0, 4.0, 1.0, 0.0])
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=1e-5, max_iters=20000)
        sc = ctx.branch_scores(parent.obj)
        st = ctx.get_batch(want_x=False, want_y=False)["status"]
    assert st[0] == P.STATUS_INFEASIBLE_BOUNDS
    assert sc["gain"][0] == math.inf and sc["score"][0] == math.inf and sc["score"][1] == math.inf
    assert math.isnan(sc["score"][2]) and math.isnan(sc["gain"][3]) and math.isnan(sc["score"][3])
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D)
        with pytest.raises(P.PdlpbError) as e:
            ctx.branch_scores(parent.obj)
        assert e.value.code == P.ESTATE
        ctx.solve(tol=1e-5, max_iters=20000)
        with pytest.raises(P.PdlpbError) as e:
            ctx.branch_scores(parent.obj, mu=1.5)
        assert e.value.code == P.EINVAL


def test_strict_dual_tolerance_matches_oracle(P):
    """With free variables the dual residual is nonzero; a strict dual epsilon
    changes when the LP stops, identically on both sides."""
    A = sp.csr_matrix(np.array([[1.0, 1.0, 1.0], [1.0, -1.0, 0.0]]))
    c = np.array([1.0, 2.0, 0.5])
    b = np.array([3.0, 0.5])
    sense = np.frombuffer(b"EL", dtype=np.uint8)
    xl = np.array([0.0, -np.inf, 0.0])
    xu = np.array([np.inf, np.inf, 4.0])
    lp = O.from_arrays(2, 3, A.indptr, A.indices, A.data, c, b, sense, xl, xu)
    eta = O.step_size(lp.A)
    for dual_tol in (-1.0, 1e-9):
        ores = oracle_run(lp, eta, 1e-3, 400000, dual_tol=None if dual_tol < 0 else dual_tol)
        ctx = P.Context(2, 3, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data, c, b,
                        sense, xl, xu, step_size=eta, dual_tol=dual_tol)
        with ctx:
            ctx.set_batch(deltas([BASE], [0], [0.0]))
            ctx.solve(tol=1e-3, max_iters=400000)
            r = ctx.get(0)
        assert r["status"] == ores.status == P.STATUS_OPTIMAL
        assert r["iters"] == ores.iters
        assert np.linalg.norm(r["x"] - ores.x) <= RTOL * max(np.linalg.norm(ores.x), 1.0)
        if dual_tol > 0:
            assert r["kkt"][2] <= dual_tol
