"""Pins for the stopping tests between evaluations (option stop_every = S).

The schedule of Section 4 is left open by the paper; the reading here tests
eq:stopping at z~ every S iterations between the evaluations that hold the
residual, restart and infeasibility tests.  What it must and must not change:

* the iterates: a run with S stops at some iteration K; the run without S,
  capped at K iterations, returns the same z~, the same Halpern iterate and
  the same restart log, bit for bit;
* the stop: K - 1 is a multiple of S (or of C), the KKT measures at K meet the
  tolerance, and at the previous test point (K - S iterations) they did not;
* it never stops later than the run without S.
"""
import numpy as np
import pytest

import oracle as O
from workloads import make_cfg2, choose_fractional, fsb_deltas, seed_for

C, S, TOL = 32, 8, 1e-4


@pytest.fixture(scope="module")
def family():
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    root = O.solve(lp, O.Options(tol=1e-7, step_size=eta))
    D = fsb_deltas(root.x, choose_fractional(root.x, 6, seed_for(2, 31)))
    return lp, eta, root, D


def _run(lp, eta, root, tol, K, stop_every):
    opt = O.Options(tol=tol, max_iters=K, step_size=eta, eval_every=C, stop_every=stop_every)
    return O.solve(lp, opt, x_init=root.x, y_init=root.y, w_init=root.w)


def test_stop_tests_change_only_when_the_lp_stops(family):
    lp, eta, root, D = family
    earlier = 0
    for d in D:
        lpj = O.apply_delta(lp, int(d["kind"]), int(d["var"]), float(d["value"]))
        plain = _run(lpj, eta, root, TOL, 100000, 0)
        fast = _run(lpj, eta, root, TOL, 100000, S)
        assert plain.status == fast.status == O.OPTIMAL
        K = fast.iters
        assert K <= plain.iters
        assert (K - 1) % S == 0
        earlier += K < plain.iters
        # the same trajectory: the run without the tests, capped at K iterations
        capped = _run(lpj, eta, root, 0.0, K, 0)
        assert capped.status == O.ITERATION_LIMIT and capped.iters == K
        assert capped.restarts == fast.restarts == plain.restarts[:len(fast.restarts)]
        for a, b in ((fast.x, capped.x), (fast.y, capped.y), (fast.x_iter, capped.x_iter),
                     (fast.y_iter, capped.y_iter)):
            assert np.array_equal(a, b)
        # the stop is the first test point that meets the tolerance
        assert fast.kkt.rel <= TOL
        if K - 1 >= S:
            before = _run(lpj, eta, root, 0.0, K - S, 0)
            assert before.kkt.rel > TOL
    assert earlier > 0          # on this family the tests do stop LPs sooner


def test_stop_every_must_divide_the_evaluation_interval(family):
    lp, eta, root, D = family
    for bad in (1, 3, 5, 33):
        with pytest.raises(ValueError):
            _run(lp, eta, root, TOL, 10, bad)
    # S = C is the same as no extra tests
    a = _run(lp, eta, root, TOL, 2000, C)
    b = _run(lp, eta, root, TOL, 2000, 0)
    assert a.iters == b.iters and np.array_equal(a.x, b.x)


def test_stop_tests_belong_to_the_per_lp_scope(family):
    lp, eta, root, D = family
    with pytest.raises(ValueError):
        O.solve_batch_avg([lp, lp], O.Options(eval_every=C, stop_every=S, step_size=eta))
