"""Scale covariance of the oracle's iteration (a symmetry of the LP, not a
restatement of the oracle's formulas).

Rescale an LP's data: the objective by alpha, and the variable box, the row
bounds and the right-hand side by beta.  Its solutions scale the same way
(x* -> beta x*, and by the saddle function of eq:lp_saddle the dual y* ->
alpha y*, the reduced cost r* -> alpha r*).  The restarted Halpern PDHG of
Section 4 maps the scaled LP's iterates onto the original ones exactly when
the primal weight scales by alpha / beta: then tau = eta / w scales by
beta / alpha and sigma = eta w by alpha / beta, each projection step maps
onto the original one, the fixed-point residual of eq:residual scales by
sqrt(alpha beta) (so the restart tests, which compare residuals, decide the
same), and the anchor displacements scale by beta and alpha.

This pins two readings of the paper that no formula in it fixes:
  * the initial primal weight (not stated): ||c|| / ||b|| scales by
    alpha / beta; 1, or ||b|| / ||c||, does not;
  * the primal-weight ratio of the restart update (printed ||dx|| / ||dy||,
    read as ||dy|| / ||dx||): only the latter scales by alpha / beta.
It does not pin a constant factor in the initial weight (any k ||c|| / ||b||
is covariant); that factor is a reading with parity unpinned.

With alpha and beta powers of two every scaling is exact in floating point,
so the trajectories agree to rounding of the logarithms in the weight update.
"""
import numpy as np
import pytest

import oracle as O
import oracle.pdhg as OP
from workloads import make_cfg2

ALPHA, BETA = 4.0, 0.125
K = 400


def _scaled(lp, alpha, beta):
    return O.LP(A=lp.A, c=alpha * lp.c, l=beta * lp.l, u=beta * lp.u, xl=beta * lp.xl,
                xu=beta * lp.xu, b=beta * lp.b)


@pytest.fixture(scope="module")
def lp_pair():
    lp = O.from_instance(make_cfg2(m=60, n=150))
    return lp, _scaled(lp, ALPHA, BETA), O.step_size(lp.A)


def _run(lp, eta, **kw):
    return O.solve(lp, O.Options(tol=0.0, max_iters=K, step_size=eta, **kw))


def _discrepancy(a, b):
    """Largest relative distance between b and the scaled image of a."""
    ex = np.max(np.abs(b.x - BETA * a.x)) / max(np.max(np.abs(BETA * a.x)), 1e-300)
    ey = np.max(np.abs(b.y - ALPHA * a.y)) / max(np.max(np.abs(ALPHA * a.y)), 1e-300)
    return max(ex, ey)


def test_initial_weight_scales_with_the_data(lp_pair):
    lp, lp2, _ = lp_pair
    w, w2 = O.initial_primal_weight(lp), O.initial_primal_weight(lp2)
    assert w2 == pytest.approx(ALPHA / BETA * w, rel=1e-15)


def test_trajectory_of_the_scaled_lp_is_the_scaled_trajectory(lp_pair):
    lp, lp2, eta = lp_pair
    a, b = _run(lp, eta), _run(lp2, eta)
    assert len(a.restarts) >= 2          # the weight update is exercised
    assert a.restarts == b.restarts and a.iters == b.iters
    assert b.w == pytest.approx(ALPHA / BETA * a.w, rel=1e-12)
    assert _discrepancy(a, b) <= 1e-10
    # the Halpern iterates too
    assert np.max(np.abs(b.x_iter - BETA * a.x_iter)) <= 1e-10 * np.max(np.abs(BETA * a.x_iter))
    assert np.max(np.abs(b.y_iter - ALPHA * a.y_iter)) <= 1e-10 * np.max(np.abs(ALPHA * a.y_iter))


@pytest.mark.parametrize("wrong", [lambda lp: 1.0,
                                   lambda lp: float(np.linalg.norm(lp.b) / np.linalg.norm(lp.c))])
def test_an_initial_weight_that_does_not_scale_breaks_covariance(lp_pair, monkeypatch, wrong):
    lp, lp2, eta = lp_pair
    monkeypatch.setattr(OP, "initial_primal_weight", wrong)
    a, b = _run(lp, eta), _run(lp2, eta)
    assert a.restarts != b.restarts or _discrepancy(a, b) > 1e-3


def test_the_printed_weight_ratio_breaks_covariance(lp_pair):
    lp, lp2, eta = lp_pair
    # start both at weights that scale correctly, so only the update differs
    a = O.solve(lp, O.Options(tol=0.0, max_iters=K, step_size=eta, pw_ratio="dx/dy"))
    b = O.solve(lp2, O.Options(tol=0.0, max_iters=K, step_size=eta, pw_ratio="dx/dy"))
    assert len(a.restarts) >= 1
    assert a.restarts != b.restarts or _discrepancy(a, b) > 1e-3
