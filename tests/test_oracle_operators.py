"""Pins for the reference solver's elementary operators (Sections 3-4).

Each operator is checked against an independent statement of what it must
be: a scalar minimisation for the proximal steps, a brute-force nearest point
for the projections, a hand-solved primal-dual pair for the fixed point of T,
and HiGHS duals for strong duality of the support-function dual, HiGHS optima
for its weak duality.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import minimize_scalar

import oracle as O
from tests.lp_exact import highs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "textbook_lps.json")
INF = np.inf


def _fixture_lps():
    with open(GOLDEN) as f:
        data = json.load(f)["lps"]
    out = []
    for d in data:
        A = np.array(d["A"])
        csr = sp.csr_matrix(A)
        lp = O.from_arrays(A.shape[0], A.shape[1], csr.indptr, csr.indices, csr.data, d["c"],
                           d["b"], np.frombuffer(d["sense"].encode(), dtype=np.uint8),
                           d["l"], d["u"])
        out.append((d, lp))
    return out


def test_proj_box_hand_values():
    v = np.array([-3.0, 0.5, 7.0, 2.0, -1.0])
    a = np.array([-1.0, 0.0, 0.0, -INF, -INF])
    b = np.array([1.0, 1.0, 5.0, 1.0, INF])
    np.testing.assert_array_equal(O.proj_box(v, a, b), [-1.0, 0.5, 5.0, 1.0, -1.0])


def test_support_hand_values_and_zero_times_inf():
    a = np.array([-1.0, 0.0, -INF, 2.0])
    b = np.array([3.0, INF, 4.0, 2.0])
    # sup over the box of v'z, coordinate by coordinate
    assert O.support(np.array([2.0, 0.0, 0.0, -1.0]), a, b) == 2 * 3 + 0 + 0 + (-1) * 2
    assert O.support(np.array([-2.0, -1.0, 1.0, 0.0]), a, b) == 2 + 0 + 4 + 0
    # a component pointing at an infinite side: unbounded
    assert O.support(np.array([0.0, 1.0, 0.0, 0.0]), a, b) == INF
    assert O.support(np.array([0.0, 0.0, -1.0, 0.0]), a, b) == INF


def test_support_is_sup_over_box_corners():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = rng.uniform(-3, 0, 4)
        b = a + rng.uniform(0, 3, 4)
        v = rng.standard_normal(4)
        corners = np.array(np.meshgrid(*[[a[i], b[i]] for i in range(4)])).reshape(4, -1).T
        assert math.isclose(O.support(v, a, b), float(np.max(corners @ v)), rel_tol=1e-12,
                            abs_tol=1e-12)


def test_proj_barrier_cone_is_nearest_point():
    a = np.array([-INF, 0.0, -INF, -2.0])
    b = np.array([1.0, INF, INF, 3.0])
    rng = np.random.default_rng(1)
    grid = np.linspace(-5, 5, 2001)
    for _ in range(10):
        v = rng.uniform(-4, 4, 4)
        p = O.proj_barrier_cone(v, a, b)
        for i in range(4):
            # cone coordinate sets: [0,inf), (-inf,0], {0}, R
            feas = {0: grid >= 0, 1: grid <= 0, 2: grid == 0, 3: np.ones_like(grid, bool)}[i]
            g = grid[feas]
            best = g[np.argmin(np.abs(g - v[i]))]
            assert abs(p[i] - best) <= 5e-3 + 1e-12


def _random_lp(seed, m=4, n=6, senses="ELGN"):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * (rng.random((m, n)) < 0.7)
    csr = sp.csr_matrix(A)
    b = rng.standard_normal(m)
    sense = np.array([ord(senses[i % len(senses)]) for i in range(m)], dtype=np.uint8)
    xl = rng.uniform(-2, 0, n)
    xu = xl + rng.uniform(0.5, 3, n)
    xl[0] = -INF
    xu[1] = INF
    return O.from_arrays(m, n, csr.indptr, csr.indices, csr.data, rng.standard_normal(n), b,
                         sense, xl, xu), rng


@pytest.mark.parametrize("seed", range(5))
def test_primal_step_is_proximal_minimiser(seed):
    """x~ = argmin over the box of (c + A'y)'x + ||x - x^k||^2 / (2 tau)."""
    lp, rng = _random_lp(seed)
    x = rng.standard_normal(lp.n)
    y = rng.standard_normal(lp.m)
    tau, sigma = 0.3, 0.7
    x_t, _ = O.pdhg_operator(lp, x, y, tau, sigma)
    g = lp.c + lp.A.toarray().T @ y
    for j in range(lp.n):
        lo = lp.xl[j] if np.isfinite(lp.xl[j]) else -1e3
        hi = lp.xu[j] if np.isfinite(lp.xu[j]) else 1e3
        f = lambda s: g[j] * s + (s - x[j]) ** 2 / (2 * tau)
        best = minimize_scalar(f, bounds=(lo, hi), method="bounded",
                               options={"xatol": 1e-12}).x
        assert abs(x_t[j] - best) < 1e-7


@pytest.mark.parametrize("seed", range(5))
def test_dual_step_is_proximal_maximiser(seed):
    """y~ = argmax_y' { y'(A(2x~ - x)) - phi_[l,u](y') - ||y' - y||^2 / (2 sigma) },
    solved coordinate by coordinate by a scalar search (phi restricted to the
    barrier cone, where it is finite)."""
    lp, rng = _random_lp(seed)
    x = rng.standard_normal(lp.n)
    y = rng.standard_normal(lp.m)
    tau, sigma = 0.3, 0.7
    x_t, y_t = O.pdhg_operator(lp, x, y, tau, sigma)
    v = lp.A.toarray() @ (2 * x_t - x)
    for i in range(lp.m):
        li, ui = lp.l[i], lp.u[i]
        lo = 0.0 if not np.isfinite(li) else -1e3       # barrier cone of [l_i, u_i]
        hi = 0.0 if not np.isfinite(ui) else 1e3
        if lo == hi:
            assert y_t[i] == 0.0
            continue

        def negobj(s):
            phi = (ui * s if s > 0 else 0.0) + (li * s if s < 0 else 0.0)
            return -(s * v[i] - phi - (s - y[i]) ** 2 / (2 * sigma))

        best = minimize_scalar(negobj, bounds=(lo, hi), method="bounded",
                               options={"xatol": 1e-12}).x
        assert abs(y_t[i] - best) < 1e-6


def test_dual_step_stays_in_barrier_cone_exactly():
    lp, rng = _random_lp(7, m=40, n=30, senses="LGN")
    for _ in range(20):
        _, y_t = O.pdhg_operator(lp, rng.standard_normal(lp.n) * 3, rng.standard_normal(lp.m) * 3,
                                 0.4, 0.9)
        np.testing.assert_array_equal(O.proj_barrier_cone(y_t, lp.l, lp.u), y_t)


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_hand_solved_pair_is_fixed_point_of_T(idx):
    d, lp = _fixture_lps()[idx]
    x, y = np.array(d["x"]), np.array(d["y"])
    for tau, sigma in [(0.1, 0.2), (1.0, 1.0), (3.0, 0.05)]:
        x_t, y_t = O.pdhg_operator(lp, x, y, tau, sigma)
        np.testing.assert_allclose(x_t, x, atol=1e-12)
        np.testing.assert_allclose(y_t, y, atol=1e-12)
        assert O.fixed_point_residual(lp, x, y, x_t, y_t, 1.0, 0.5) < 1e-10


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_hand_solved_pair_has_zero_kkt_and_strong_duality(idx):
    d, lp = _fixture_lps()[idx]
    k = O.kkt(lp, np.array(d["x"]), np.array(d["y"]))
    assert abs(k.obj - d["obj"]) < 1e-12
    assert abs(k.dual_obj - d["obj"]) < 1e-12
    assert k.rel < 1e-14


def test_kkt_detects_each_violation():
    d, lp = _fixture_lps()[1]
    x, y = np.array(d["x"]), np.array(d["y"])
    # primal infeasible point (equality row broken) -> primal measure grows
    k = O.kkt(lp, x + np.array([0.0, 0.5, 0.0]), y)
    assert k.primal > 0.05
    # suboptimal dual -> gap grows
    k = O.kkt(lp, x, y + np.array([0.5, 0.0]))
    assert k.gap > 0.05
    # free variables expose the dual residual: r is forced to 0 on free coordinates
    lp2 = O.LP(A=lp.A, c=lp.c, l=lp.l, u=lp.u, xl=np.full(3, -INF), xu=np.full(3, INF), b=lp.b)
    k = O.kkt(lp2, x, y)
    assert k.dual > 0.1


def test_highs_duals_give_zero_kkt_on_random_lp():
    """Strong duality of the support-function dual (eq:main_lp) at an
    independent solver's optimal pair pins the signs of y, r and phi."""
    from workloads import make_tiny
    lp = O.from_instance(make_tiny(11, m=6, n=9, senses="ELG", box=(-2.0, 3.0)))
    obj, x, y = highs(lp)
    k = O.kkt(lp, x, y)
    assert abs(k.obj - obj) < 1e-9
    assert k.rel < 1e-8
    x_t, y_t = O.pdhg_operator(lp, x, y, 0.2, 0.3)
    np.testing.assert_allclose(x_t, x, atol=1e-8)
    np.testing.assert_allclose(y_t, y, atol=1e-8)


def test_row_bounds_mapping():
    l, u = O.row_bounds(np.array([1.0, 2.0, 3.0, 4.0]), np.frombuffer(b"ELGN", dtype=np.uint8))
    np.testing.assert_array_equal(l, [1.0, -INF, 3.0, -INF])
    np.testing.assert_array_equal(u, [1.0, 2.0, INF, INF])
    with pytest.raises(ValueError):
        O.row_bounds(np.array([1.0]), np.frombuffer(b"X", dtype=np.uint8))


def test_apply_delta_kinds():
    lp, _ = _random_lp(3)
    up = O.apply_delta(lp, O.SET_LO, 2, 1.5)
    assert up.xl[2] == 1.5 and np.array_equal(up.xu, lp.xu) and up.xl[3] == lp.xl[3]
    dn = O.apply_delta(lp, O.SET_HI, 4, -0.5)
    assert dn.xu[4] == -0.5 and np.array_equal(dn.xl, lp.xl)
    ob = O.apply_delta(lp, O.OBJ_UNIT, 1, -1.0)
    assert ob.c[1] == -1.0 and np.count_nonzero(ob.c) == 1
    assert O.apply_delta(lp, O.BASE, 0, 0.0).c is lp.c



def _dual_value(lp, y, flip_aty=False):
    """The dual objective as the oracle's KKT reports it; with flip_aty, the
    same with the sign of A'y in the reduced cost flipped (a planted mistake)."""
    if not flip_aty:
        return O.kkt(lp, O.proj_box(np.zeros(lp.n), lp.xl, lp.xu), y).dual_obj
    r = O.proj_barrier_cone(-lp.c + lp.A.T @ y, lp.xl, lp.xu)
    return -(O.support(r, lp.xl, lp.xu) + O.support(y, lp.l, lp.u))


@pytest.mark.parametrize("seed", range(4))
def test_dual_objective_is_a_lower_bound(seed):
    """Weak duality: with a finite box, the dual objective at ANY dual point of
    the barrier cone is at most the LP optimum (HiGHS), and it reaches it at the
    optimal duals (checked above).  The sign of A'y flipped in the reduced cost,
    planted on the CPU, exceeds the optimum."""
    from workloads import make_tiny
    lp = O.from_instance(make_tiny(seed, m=4, n=7, senses="ELG", box=(0.0, 3.0)))
    opt, _, _ = highs(lp)
    rng = np.random.default_rng(seed)
    worst = -np.inf
    worst_planted = -np.inf
    for scale in (0.1, 1.0, 10.0, 100.0):
        for _ in range(100):
            y = O.proj_barrier_cone(rng.normal(scale=scale, size=lp.m), lp.l, lp.u)
            worst = max(worst, _dual_value(lp, y) - opt)
            worst_planted = max(worst_planted, _dual_value(lp, y, flip_aty=True) - opt)
    assert worst <= 1e-9 * (1 + abs(opt)), worst
    assert worst_planted > 1e-3, worst_planted
