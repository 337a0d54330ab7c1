"""Pins for the MIP-facing outputs (Sections 5.1, 5.2 and the OBBT experiments
of Section 6): safe OBBT bounds bracket the exact variable range found by
vertex enumeration, known tightenings happen, sub-threshold ones do not, the
box-only case reduces to its closed form, and the branching gains match exact
child optima."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle import mip as M
from tests.lp_exact import vertex_enum
from workloads import make_tiny

INF = np.inf


def _lp(A, b, sense, c, xl, xu):
    A = sp.csr_matrix(np.array(A, dtype=float))
    return O.from_arrays(A.shape[0], A.shape[1], A.indptr, A.indices, A.data, c, b,
                         np.frombuffer(sense.encode(), dtype=np.uint8), xl, xu)


def _obbt(lp, tol=1e-9, dual_tol=M.OBBT_DUAL_TOL):
    """Solve min x_v and min -x_v for every v; return (vars, signs, results)."""
    var, sign, res = [], [], []
    opt = O.Options(tol=tol, dual_tol=dual_tol, max_iters=400000)
    for v in range(lp.n):
        for s in (1.0, -1.0):
            var.append(v)
            sign.append(s)
            res.append(O.solve(O.apply_delta(lp, O.OBJ_UNIT, v, s), opt))
    return var, sign, res


@pytest.mark.parametrize("seed", range(4))
def test_safe_bounds_bracket_the_exact_range(seed):
    lp = O.from_instance(make_tiny(seed, m=3, n=4, senses="ELG", box=(0.0, 4.0)))
    A = lp.A.toarray()
    var, sign, res = _obbt(lp)
    for v, s, r in zip(var, sign, res):
        assert r.status == O.OPTIMAL
        c = np.zeros(lp.n)
        c[v] = s
        exact, _ = vertex_enum(A, lp.l, lp.u, lp.xl, lp.xu, c)
        b = M.obbt_bound(r, s, M.OBBT_DUAL_TOL)
        if s > 0:               # lower bound on min x_v
            assert b <= exact + 1e-12
            assert exact - b <= 1e-6
        else:                   # upper bound on max x_v = -exact
            assert b >= -exact - 1e-12
            assert b - (-exact) <= 1e-6


def test_known_tightening():
    # x1 + x2 <= 1 with x in [0, 10]^2: both upper bounds fall to 1, lower stay 0
    lp = _lp([[1.0, 1.0]], [1.0], "L", [0.0, 0.0], [0.0, 0.0], [10.0, 10.0])
    var, sign, res = _obbt(lp)
    t = M.obbt_tighten(lp.xl, lp.xu, var, sign, res)
    assert not t.infeasible
    assert t.changed == 2
    np.testing.assert_array_equal(t.xl, [0.0, 0.0])
    assert np.all(t.xu >= 1.0) and np.all(t.xu <= 1.0 + 1e-6)


@pytest.mark.parametrize("cap,moves", [(10.0 - 5e-5, False), (10.0 - 2e-4, True)])
def test_improvement_threshold(cap, moves):
    # x1 <= cap as a row; the OBBT upper bound of x1 moves only if 10 - cap > 1e-4
    lp = _lp([[1.0, 0.0]], [cap], "L", [0.0, 0.0], [0.0, 0.0], [10.0, 10.0])
    var, sign, res = _obbt(lp)
    t = M.obbt_tighten(lp.xl, lp.xu, var, sign, res)
    assert (t.xu[0] < 10.0) == moves
    if moves:
        assert cap <= t.xu[0] <= cap + 1e-6
    assert t.xu[1] == 10.0 and np.all(t.xl == 0.0)


def test_box_only_closed_form():
    # free rows: min x_v is its lower bound, the dual objective equals it, and
    # the shifted bound sits Delta below it, so nothing is tightened
    lp = _lp([[1.0, 2.0, -1.0]], [0.0], "N", [0.0, 0.0, 0.0], [-1.0, 2.0, 0.5], [3.0, 5.0, 4.0])
    var, sign, res = _obbt(lp)
    for v, s, r in zip(var, sign, res):
        exact = lp.xl[v] if s > 0 else -lp.xu[v]      # min s * x_v
        assert r.kkt.dual_obj == pytest.approx(exact, abs=1e-12)
        delta = M.OBBT_DUAL_TOL * (1.0 + abs(exact) + abs(exact))
        want = exact - delta if s > 0 else -exact + delta
        assert M.obbt_bound(r, s, M.OBBT_DUAL_TOL) == pytest.approx(want, abs=1e-14)
    t = M.obbt_tighten(lp.xl, lp.xu, var, sign, res)
    assert t.changed == 0
    np.testing.assert_array_equal(t.xl, lp.xl)
    np.testing.assert_array_equal(t.xu, lp.xu)


def test_infeasible_set_is_reported():
    lp = _lp([[1.0, 1.0]], [5.0], "E", [0.0, 0.0], [0.0, 0.0], [1.0, 1.0])
    var, sign, res = _obbt(lp, tol=1e-8, dual_tol=None)
    t = M.obbt_tighten(lp.xl, lp.xu, var, sign, res)
    assert t.infeasible and t.changed == 0


def test_unconverged_lp_gives_no_bound():
    lp = _lp([[1.0, 1.0]], [1.0], "L", [0.0, 0.0], [0.0, 0.0], [10.0, 10.0])
    r = O.solve(O.apply_delta(lp, O.OBJ_UNIT, 0, -1.0), O.Options(tol=1e-12, max_iters=3))
    assert r.status == O.ITERATION_LIMIT
    assert M.obbt_bound(r, -1.0, M.OBBT_DUAL_TOL) is None
    t = M.obbt_tighten(lp.xl, lp.xu, [0], [-1.0], [r])
    assert t.changed == 0


def test_dual_tolerance_is_enforced():
    """With free variables the dual residual is not identically zero; a strict
    dual epsilon makes the solver stop only once that residual meets it."""
    lp = _lp([[1.0, 1.0, 1.0], [1.0, -1.0, 0.0]], [3.0, 0.5], "EL",
             [1.0, 2.0, 0.5], [0.0, -INF, 0.0], [INF, INF, 4.0])
    loose = O.solve(lp, O.Options(tol=1e-3))
    strict = O.solve(lp, O.Options(tol=1e-3, dual_tol=1e-9, max_iters=400000))
    assert loose.status == strict.status == O.OPTIMAL
    assert strict.kkt.dual <= 1e-9
    assert strict.kkt.gap <= 1e-3 and strict.kkt.primal <= 1e-3
    assert strict.iters >= loose.iters


def test_branch_score_formula():
    assert M.branch_score(1.0, 4.0) == pytest.approx(5.0 / 6.0 + 4.0 / 6.0)
    assert M.branch_score(4.0, 1.0) == M.branch_score(1.0, 4.0)
    assert M.branch_score(0.0, 0.0) == 0.0
    assert M.branch_score(math.inf, 2.0) == math.inf
    assert math.isnan(M.branch_score(math.nan, 2.0))
    assert M.branch_score(2.0, 3.0, mu=0.0) == 2.0 and M.branch_score(2.0, 3.0, mu=1.0) == 3.0


@pytest.mark.parametrize("seed", range(3))
def test_branch_gains_match_exact_children(seed):
    lp = O.from_instance(make_tiny(seed, m=3, n=4, senses="ELG", box=(0.0, 4.0)))
    A = lp.A.toarray()
    parent_exact, xp = vertex_enum(A, lp.l, lp.u, lp.xl, lp.xu, lp.c)
    parent = O.solve(lp, O.Options(tol=1e-10, max_iters=400000))
    assert parent.obj == pytest.approx(parent_exact, abs=1e-6)
    frac = [j for j in range(lp.n) if 0.05 < parent.x[j] - math.floor(parent.x[j]) < 0.95]
    for j in frac:
        up_lp = O.apply_delta(lp, O.SET_LO, j, math.ceil(parent.x[j]))
        dn_lp = O.apply_delta(lp, O.SET_HI, j, math.floor(parent.x[j]))
        gains = []
        for ch in (dn_lp, up_lp):
            ex, _ = vertex_enum(A, ch.l, ch.u, ch.xl, ch.xu, ch.c)
            r = O.solve(ch, O.Options(tol=1e-10, max_iters=400000))
            g = M.branch_gain(r, parent.obj)
            if math.isinf(ex):
                assert r.status == O.PRIMAL_INFEASIBLE and g == math.inf
            else:
                assert g == pytest.approx(max(ex - parent_exact, 0.0), abs=1e-5)
            gains.append(g)
        s = M.branch_score(*gains)
        assert s >= min(gains) - 1e-12
