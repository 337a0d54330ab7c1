"""Pins for the fixed-point residual (eq:residual), the step size, the restart
rule and the primal-weight smoothing (Section 4)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from workloads import make_tiny, make_cfg1


def _lp(seed, m=5, n=7):
    return O.from_instance(make_tiny(seed, m=m, n=n, senses="ELG", box=(-1.0, 3.0)))


def _metric_inner(lp, w, eta, s, z1, z2):
    """<z1, z2>_M for M = [[(w/eta) I, s A'], [s A, 1/(eta w) I]], built as a dense matrix."""
    A = lp.A.toarray()
    n, m = lp.n, lp.m
    M = np.block([[(w / eta) * np.eye(n), s * A.T], [s * A, (1 / (eta * w)) * np.eye(m)]])
    return float(z1 @ M @ z2)


@pytest.mark.parametrize("seed", range(4))
def test_T_firmly_nonexpansive_in_the_chosen_metric(seed):
    """<Tz1 - Tz2, z1 - z2>_M >= ||Tz1 - Tz2||_M^2 for all pairs, with the cross
    term sign -1.  This is the property that makes r(z) a meaningful progress
    measure for the Halpern iteration; the sign printed in eq:residual (+1)
    violates it, which is why the default reading flips it."""
    lp = _lp(seed)
    eta = O.step_size(lp.A)
    rng = np.random.default_rng(100 + seed)
    worst_chosen, worst_literal = np.inf, np.inf
    for _ in range(400):
        w = float(np.exp(rng.uniform(-2, 2)))
        z1 = rng.standard_normal(lp.n + lp.m) * 3
        z2 = rng.standard_normal(lp.n + lp.m) * 3
        t1 = np.concatenate(O.pdhg_operator(lp, z1[:lp.n], z1[lp.n:], eta / w, eta * w))
        t2 = np.concatenate(O.pdhg_operator(lp, z2[:lp.n], z2[lp.n:], eta / w, eta * w))
        dT, dz = t1 - t2, z1 - z2
        for s, ref in ((-1.0, "c"), (1.0, "l")):
            nz = _metric_inner(lp, w, eta, s, dz, dz)
            val = (_metric_inner(lp, w, eta, s, dT, dz) - _metric_inner(lp, w, eta, s, dT, dT)) / nz
            if ref == "c":
                worst_chosen = min(worst_chosen, val)
            else:
                worst_literal = min(worst_literal, val)
    assert worst_chosen >= -1e-10
    assert worst_literal < -1e-3


def test_residual_equals_metric_norm_and_vanishes_at_fixed_point():
    lp = _lp(3)
    eta = O.step_size(lp.A)
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(lp.n), rng.standard_normal(lp.m)
    w = 0.7
    xt, yt = O.pdhg_operator(lp, x, y, eta / w, eta * w)
    d = np.concatenate([xt - x, yt - y])
    r = O.fixed_point_residual(lp, x, y, xt, yt, w, eta)
    assert math.isclose(r, math.sqrt(_metric_inner(lp, w, eta, -1.0, d, d)), rel_tol=1e-12)
    # M is positive definite when eta ||A|| < 1: r^2 >= 0 for random displacements
    for _ in range(100):
        d = rng.standard_normal(lp.n + lp.m)
        assert _metric_inner(lp, w, eta, -1.0, d, d) > 0
    # at an optimal pair the residual is zero
    from tests.lp_exact import highs
    _, xs, ys = highs(lp)
    xt, yt = O.pdhg_operator(lp, xs, ys, eta / w, eta * w)
    assert O.fixed_point_residual(lp, xs, ys, xt, yt, w, eta) < 1e-7


@pytest.mark.parametrize("seed", range(3))
def test_opnorm_matches_dense_two_norm(seed):
    rng = np.random.default_rng(seed)
    A = sp.random(30, 45, density=0.2, random_state=seed, data_rvs=rng.standard_normal).tocsr()
    assert math.isclose(O.opnorm(A), np.linalg.norm(A.toarray(), 2), rel_tol=1e-9)


def test_opnorm_special_cases():
    assert O.opnorm(sp.csr_matrix((4, 6))) == 0.0
    assert O.step_size(sp.csr_matrix((4, 6))) == 1.0
    D = sp.diags([1.0, -7.0, 3.0]).tocsr()
    assert math.isclose(O.opnorm(D), 7.0, rel_tol=1e-12)
    lp = O.from_instance(make_cfg1())
    assert math.isclose(O.opnorm(lp.A), np.linalg.norm(lp.A.toarray(), 2), rel_tol=1e-9)
    assert math.isclose(O.step_size(lp.A) * np.linalg.norm(lp.A.toarray(), 2), 0.998, rel_tol=1e-9)


def test_restart_conditions_hand_cases():
    bs, bn, ba = 0.2, 0.8, 0.36
    # sufficient decay: r <= 0.2 r0
    assert O.restart_due(0.19, 1.0, 0.5, 10, 100, bs, bn, ba)
    assert O.restart_due(0.2, 1.0, 0.1, 10, 100, bs, bn, ba)
    # necessary decay without progress: r <= 0.8 r0 and r > r_prev
    assert O.restart_due(0.7, 1.0, 0.6, 10, 100, bs, bn, ba)
    assert not O.restart_due(0.7, 1.0, 0.75, 10, 100, bs, bn, ba)    # still progressing
    assert not O.restart_due(0.85, 1.0, 0.6, 10, 100, bs, bn, ba)    # not enough decay
    assert not O.restart_due(0.7, 1.0, None, 10, 100, bs, bn, ba)    # no previous evaluation
    # artificial: k > 0.36 t
    assert O.restart_due(0.9, 1.0, 0.95, 37, 100, bs, bn, ba)
    assert not O.restart_due(0.9, 1.0, 0.95, 36, 100, bs, bn, ba)


def test_primal_weight_smoothing_closed_form():
    # exp(theta log d + (1-theta) log w) = d^theta w^(1-theta), d = ||dy|| / ||dx||
    w = O.smoothed_primal_weight(dx_norm=2.0, dy_norm=8.0, w=0.25, theta=0.5)
    assert math.isclose(w, math.sqrt(4.0 * 0.25), rel_tol=1e-14)
    w = O.smoothed_primal_weight(2.0, 8.0, 0.25, 0.3)
    assert math.isclose(w, 4.0 ** 0.3 * 0.25 ** 0.7, rel_tol=1e-14)
    # literal ratio of the printed formula
    w = O.smoothed_primal_weight(2.0, 8.0, 0.25, 0.5, ratio="dx/dy")
    assert math.isclose(w, math.sqrt(0.25 * 0.25), rel_tol=1e-14)
    # d not finite (a zero displacement): weight kept
    assert O.smoothed_primal_weight(0.0, 3.0, 0.4, 0.5) == 0.4
    assert O.smoothed_primal_weight(3.0, 0.0, 0.4, 0.5) == 0.4
    assert O.smoothed_primal_weight(3.0, 2.0, 0.4, 1.0) == pytest.approx(2.0 / 3.0, rel=1e-14)


def test_initial_primal_weight():
    lp = O.from_instance(make_tiny(1))
    assert math.isclose(O.initial_primal_weight(lp),
                        np.linalg.norm(lp.c) / np.linalg.norm(lp.b), rel_tol=1e-14)
    lp.c = np.zeros(lp.n)
    assert O.initial_primal_weight(lp) == 1.0


def test_opnorm_when_constant_vector_is_in_null_space():
    A = sp.csr_matrix(np.array([[1.0, -1.0], [2.0, -2.0]]))
    assert math.isclose(O.opnorm(A), np.linalg.norm(A.toarray(), 2), rel_tol=1e-12)


def _log_imbalance(w, dx, dy, eta=0.7):
    """log of the ratio of the two diagonal terms of the residual metric,
    (w/eta) ||dx||^2 against ||dy||^2 / (eta w)."""
    return math.log((w / eta) * dx * dx) - math.log(dy * dy / (eta * w))


@pytest.mark.parametrize("seed", range(5))
def test_primal_weight_update_balances_the_metric(seed):
    """The weight update (Section 4) exists to balance the primal and dual
    parts of the residual metric: with the ratio ||dy|| / ||dx|| (reading R2),
    smoothing with theta shrinks their log-imbalance by the factor 1 - theta,
    and theta = 1 balances them exactly.  The printed ratio ||dx|| / ||dy||, or
    the two smoothing weights swapped, breaks this."""
    rng = np.random.default_rng(seed)
    dx, dy = np.exp(rng.uniform(-3, 3, size=2))
    w0 = float(np.exp(rng.uniform(-3, 3)))
    before = _log_imbalance(w0, dx, dy)
    for theta in (0.0, 0.3, 0.5, 1.0):
        after = _log_imbalance(O.smoothed_primal_weight(dx, dy, w0, theta), dx, dy)
        assert math.isclose(after, (1.0 - theta) * before, rel_tol=1e-9, abs_tol=1e-9)
    # planted mistakes, on the CPU: the printed ratio, and the weights swapped
    printed = _log_imbalance(O.smoothed_primal_weight(dx, dy, w0, 1.0, ratio="dx/dy"), dx, dy)
    assert abs(printed) > 1e-3
    swapped = w0 ** 0.3 * (dy / dx) ** 0.7                 # theta applied to the old weight
    assert not math.isclose(_log_imbalance(swapped, dx, dy), 0.7 * before, rel_tol=1e-6)
