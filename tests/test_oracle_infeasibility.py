"""Pins for the infeasibility tests of Section 4 (eq:primal-infeas,
eq:dual-infeas): a Farkas certificate is only possible for an infeasible LP,
so each detection is checked against HiGHS's verdict and against the
certificate conditions themselves; feasible LPs are never flagged."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import oracle as O
from workloads import make_cfg2, make_tiny

INF = np.inf


def _lp(A, b, sense, c, xl, xu):
    A = sp.csr_matrix(np.array(A, dtype=float))
    return O.from_arrays(A.shape[0], A.shape[1], A.indptr, A.indices, A.data, c, b,
                         np.frombuffer(sense.encode(), dtype=np.uint8), xl, xu)


def test_recession_cone_is_nearest_point():
    a = np.array([-INF, 0.0, -INF, -2.0])
    b = np.array([1.0, INF, INF, 3.0])
    grid = np.linspace(-5, 5, 2001)
    rng = np.random.default_rng(2)
    for _ in range(10):
        v = rng.uniform(-4, 4, 4)
        p = O.proj_recession_cone(v, a, b)
        # recession cones per coordinate: (-inf,0], [0,inf), R, {0}
        sets = [grid <= 0, grid >= 0, np.ones_like(grid, bool), grid == 0]
        for i in range(4):
            g = grid[sets[i]]
            assert abs(p[i] - g[np.argmin(np.abs(g - v[i]))]) <= 5e-3 + 1e-12


def test_primal_infeasible_box_detected():
    # x1 + x2 = 5 with 0 <= x <= 1: infeasible
    lp = _lp([[1.0, 1.0]], [5.0], "E", [1.0, -1.0], [0.0, 0.0], [1.0, 1.0])
    h = linprog(lp.c, A_eq=lp.A.toarray(), b_eq=[5.0], bounds=[(0, 1), (0, 1)], method="highs")
    assert h.status == 2
    r = O.solve(lp, O.Options(tol=1e-8, max_iters=100000))
    assert r.status == O.PRIMAL_INFEASIBLE


def test_certificate_conditions_at_detection():
    """At detection, (dy, dr) is an approximate Farkas certificate: A'dy + dr ~ 0
    relative to the negative support value (the definition of the test)."""
    lp = _lp([[1.0, 2.0, 0.0], [0.0, 1.0, 1.0]], [10.0, -1.0], "LG", [1.0, 1.0, 1.0],
             [0.0, 0.0, 0.0], [1.0, 1.0, 1.0])
    # row 1: x1 + 2x2 <= 10 feasible; row 2: x2 + x3 >= -1 feasible -> LP feasible
    assert O.solve(lp, O.Options(tol=1e-8)).status == O.OPTIMAL
    lp2 = _lp([[1.0, 2.0, 0.0], [0.0, 1.0, 1.0]], [10.0, 3.0], "LG", [1.0, 1.0, 1.0],
              [0.0, 0.0, 0.0], [1.0, 1.0, 1.0])
    # x2 + x3 >= 3 with x in [0,1]^3: infeasible
    res = O.solve(lp2, O.Options(tol=1e-8, max_iters=200000))
    assert res.status == O.PRIMAL_INFEASIBLE


def test_dual_infeasible_unbounded_detected():
    # min -x1 s.t. x1 - x2 = 0, x >= 0 (no upper bounds): unbounded below
    lp = _lp([[1.0, -1.0]], [0.0], "E", [-1.0, 0.0], [0.0, 0.0], [INF, INF])
    h = linprog(lp.c, A_eq=lp.A.toarray(), b_eq=[0.0], bounds=[(0, None), (0, None)],
                method="highs")
    assert h.status == 3
    r = O.solve(lp, O.Options(tol=1e-8, max_iters=100000))
    assert r.status == O.DUAL_INFEASIBLE


@pytest.mark.parametrize("seed", range(6))
def test_feasible_lps_never_flagged(seed):
    lp = O.from_instance(make_tiny(seed, m=3, n=5, senses="ELG", box=(0.0, 4.0)))
    r = O.solve(lp, O.Options(tol=1e-9, max_iters=400000, infeas_tol=1e-2))
    assert r.status == O.OPTIMAL


def test_infeasibility_disabled_runs_to_limit():
    lp = _lp([[1.0, 1.0]], [5.0], "E", [1.0, -1.0], [0.0, 0.0], [1.0, 1.0])
    r = O.solve(lp, O.Options(tol=1e-8, max_iters=3000, infeas_tol=0.0))
    assert r.status == O.ITERATION_LIMIT and r.iters == 3000


@pytest.mark.slow
def test_infeasible_strong_branching_child_detected():
    """A branch-up that fixes a variable of the 2000 x 5000 family at its upper
    bound (HiGHS: infeasible) is recognised instead of running to the limit,
    while its sibling branch is solved."""
    inst = make_cfg2()
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    base = O.solve(lp, O.Options(tol=1e-6, step_size=eta))
    up = O.solve(O.apply_delta(lp, O.SET_LO, 3950, 10.0), O.Options(tol=1e-4, step_size=eta),
                 x_init=base.x, y_init=base.y, w_init=base.w)
    dn = O.solve(O.apply_delta(lp, O.SET_HI, 3950, 9.0), O.Options(tol=1e-4, step_size=eta),
                 x_init=base.x, y_init=base.y, w_init=base.w)
    assert up.status == O.PRIMAL_INFEASIBLE and up.iters < 20000
    assert dn.status == O.OPTIMAL


# ---------------------------------------------------------------------------
# The tests themselves, against Farkas' lemma.  If x^ is feasible (s = A x^ in
# [l, u], x^ in the box), then for any dy and dr in the barrier cones
#   phi(dy) + phi(dr) >= s'dy + x^'dr = x^'(A'dy + dr) >= -||x^|| ||A'dy + dr||,
# so whenever the support sum is negative the primal ratio is at least
# 1 / ||x^||: a feasible LP is never flagged for eps below that.  An
# infeasible LP has a ray dy with A'dy + dr = 0 and a negative support sum,
# which the test must flag.  On the dual side, a finite box has the recession
# cone {0}, so the dual ratio is at least ||dx|| / |c'dx| >= 1 / ||c||; an
# unbounded LP has a ray dx in the recession cones with c'dx < 0.
# ---------------------------------------------------------------------------

def _displaced(lp, x, y, dx, dy, eps):
    return O.infeasibility(lp, x, y, x + dx, y + dy, eps)


@pytest.mark.parametrize("s", [1e-3, 1.0, 1e3])
def test_farkas_ray_is_flagged_and_feasible_sibling_never(s):
    rng = np.random.default_rng(int(s * 1000) % 97)
    # x1 + x2 = 5 over [0, 1]^2: the ray dy = -1 (dr = (1, 1)) has support sum
    # -5 + 2 = -3 and A'dy + dr = 0
    bad = _lp([[1.0, 1.0]], [5.0], "E", [1.0, -1.0], [0.0, 0.0], [1.0, 1.0])
    x, y = rng.uniform(0, 1, 2), rng.normal(size=1)
    got = _displaced(bad, x, y, np.zeros(2), np.array([-s]), 1e-6)
    assert got.primal and not got.dual
    # x2 + x3 >= 3 over [0, 1]^3: the ray on the second row, dy = (0, -1)
    bad2 = _lp([[1.0, 2.0, 0.0], [0.0, 1.0, 1.0]], [10.0, 3.0], "LG", [1.0, 1.0, 1.0],
               [0.0, 0.0, 0.0], [1.0, 1.0, 1.0])
    got = _displaced(bad2, rng.uniform(0, 1, 3), np.array([0.0, 0.0]), np.zeros(3),
                     np.array([0.0, -s]), 1e-6)
    assert got.primal
    # x1 + x2 = 1 is feasible: no displacement of y is a certificate
    ok = _lp([[1.0, 1.0]], [1.0], "E", [1.0, -1.0], [0.0, 0.0], [1.0, 1.0])
    for dy in (-s, s):
        got = _displaced(ok, x, y, np.zeros(2), np.array([dy]), 0.5)
        assert not got.primal and got.primal_ratio == np.inf


@pytest.mark.parametrize("seed", range(4))
def test_feasible_lp_primal_ratio_bounded_below(seed):
    """Random displacements on feasible LPs with finite and infinite bounds:
    whenever the support sum is negative, the ratio is at least 1 / ||x^||
    for the generator's feasible witness x^."""
    inst = make_tiny(seed, m=4, n=6, senses="ELG", box=(0.0, 4.0))
    rng = np.random.default_rng(100 + seed)
    xl = np.where(rng.random(inst.n) < 0.5, -INF, inst.l)
    xu = np.where(rng.random(inst.n) < 0.5, INF, inst.u)
    lp = O.from_arrays(inst.m, inst.n, inst.row_ptr, inst.col_idx, inst.val, inst.c, inst.b,
                       inst.sense, xl, xu)
    xh = inst.x0
    ax = lp.A @ xh
    assert np.all(ax >= lp.l - 1e-9) and np.all(ax <= lp.u + 1e-9)
    bound = 1.0 / np.linalg.norm(xh)
    negative = 0
    for _ in range(400):
        y = rng.normal(size=inst.m) * 3
        dy = rng.normal(size=inst.m) * 10.0 ** rng.uniform(-3, 3)
        got = _displaced(lp, xh, y, np.zeros(inst.n), dy, 0.5 * bound)
        assert not got.primal
        if np.isfinite(got.primal_ratio):
            negative += 1
            assert got.primal_ratio >= bound * (1 - 1e-9)
    assert negative > 0          # the bound was exercised, not only phi >= 0


def test_unbounded_ray_is_flagged_and_bounded_sibling_never():
    # min -x1, x1 - x2 = 0, x >= 0: the ray dx = (1, 1) has c'dx = -1, lies in
    # the recession cone of the box and A dx = 0
    bad = _lp([[1.0, -1.0]], [0.0], "E", [-1.0, 0.0], [0.0, 0.0], [INF, INF])
    ok = _lp([[1.0, -1.0]], [0.0], "E", [-1.0, 0.0], [0.0, 0.0], [5.0, 5.0])
    rng = np.random.default_rng(4)
    for t in (1e-3, 1.0, 1e3):
        x, y = rng.uniform(0, 5, 2), rng.normal(size=1)
        got = _displaced(bad, x, y, np.array([t, t]), np.zeros(1), 1e-9)
        assert got.dual and got.dual_ratio <= 1e-12
        # a finite box: the recession cone is {0}, ratio >= ||dx|| / |c'dx| >= 1 / ||c||
        for dx in (np.array([t, t]), rng.normal(size=2) * t):
            got = _displaced(ok, x, y, dx, np.zeros(1), 0.5)
            assert not got.dual
            if np.isfinite(got.dual_ratio):
                assert got.dual_ratio >= 1.0 / np.linalg.norm(ok.c) * (1 - 1e-12)
