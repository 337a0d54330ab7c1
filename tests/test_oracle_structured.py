"""Structured 0/1 LP relaxations (set covering, facility location): the
generators' witness points are feasible, and the reference solver reaches the
optimum HiGHS reports on small members of each family."""
import numpy as np
import pytest

import oracle as O
from tests.lp_exact import highs
from workloads import make_setcover, make_facility


def _feasible(inst, x, tol=1e-12):
    lp = O.from_instance(inst)
    ax = lp.A @ x
    return (np.all(ax >= lp.l - tol) and np.all(ax <= lp.u + tol) and np.all(x >= lp.xl)
            and np.all(x <= lp.xu))


@pytest.mark.parametrize("inst", [make_setcover(0, m=40, n=80, k=4), make_setcover(1, m=60, n=50, k=3),
                                  make_facility(0, F=5, C=20, k=3), make_facility(1, F=8, C=15, k=4)],
                         ids=["cover40x80", "cover60x50", "facility5x20", "facility8x15"])
def test_structured_optimum_matches_highs(inst):
    assert _feasible(inst, inst.x0)
    lp = O.from_instance(inst)
    exact, _, _ = highs(lp)
    r = O.solve(lp, O.Options(tol=1e-8, max_iters=400000))
    assert r.status == O.OPTIMAL
    assert r.obj == pytest.approx(exact, rel=1e-6, abs=1e-6)
    # a relaxation of a 0/1 problem: some optimal values are fractional
    frac = np.abs(r.x - np.round(r.x)) > 1e-3
    assert _feasible(inst, np.clip(r.x, lp.xl, lp.xu), tol=1e-5)
    print(f"{inst.name}: obj {r.obj:.6f} iters {r.iters} fractional {frac.sum()}")
