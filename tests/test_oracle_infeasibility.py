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
