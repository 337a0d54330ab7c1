"""Diagonal preconditioning through the C ABI against the oracle's scaled
solve: the scaling vectors, iterates after a fixed iteration count, converged
statuses and iteration counts, warm starts and results in the caller's
coordinates, and serving with a scaled context."""
import numpy as np
import pytest

import oracle as O
from oracle import scaling as S
from tests.gpu_common import make_ctx, lp_for, rel_err, elem_err, ITER_RTOL
from workloads import make_badly_scaled, choose_fractional, fsb_deltas, obbt_deltas, choose_vars

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


@pytest.fixture(scope="module")
def setup():
    inst = make_badly_scaled()
    lp = O.from_instance(inst)
    dr, dc = S.scaling(lp.A)
    eta = O.step_size(S.scale_lp(lp, dr, dc).A)
    root, xr, yr = S.solve_scaled(lp, O.Options(tol=1e-6, step_size=eta), dr, dc)
    assert root.status == O.OPTIMAL
    D = fsb_deltas(xr, choose_fractional(xr, 6, seed=3))
    return inst, lp, dr, dc, eta, root, xr, yr, D


def test_scaling_vectors_match_oracle(P, setup):
    inst, lp, dr, dc = setup[:4]
    with make_ctx(inst, scaling=1) as ctx:
        gr, gc = ctx.scaling()
    np.testing.assert_allclose(gr, dr, rtol=1e-13)
    np.testing.assert_allclose(gc, dc, rtol=1e-13)
    with make_ctx(inst) as ctx:
        gr, gc = ctx.scaling()
    assert np.all(gr == 1.0) and np.all(gc == 1.0)


@pytest.mark.parametrize("K", [1, 65, 300])
def test_fixed_iterations_match_oracle(P, setup, K):
    inst, lp, dr, dc, eta, root, xr, yr, D = setup
    with make_ctx(inst, eta, scaling=1) as ctx:
        ctx.set_batch(D, x_warm=xr, y_warm=yr, w_warm=np.full(len(D), root.w))
        ctx.solve(tol=0.0, max_iters=K)
        got = [ctx.get(j) for j in range(len(D))]
    for j, d in enumerate(D):
        r, x, y = S.solve_scaled(lp_for(lp, d), O.Options(tol=0.0, max_iters=K, step_size=eta),
                                 dr, dc, x_init=xr, y_init=yr, w_init=root.w)
        assert got[j]["iters"] == r.iters == K
        assert rel_err(got[j]["x"], x) <= ITER_RTOL and rel_err(got[j]["y"], y) <= ITER_RTOL, j
        assert elem_err(got[j]["x"], x) <= ITER_RTOL and elem_err(got[j]["y"], y) <= ITER_RTOL, j


@pytest.mark.parametrize("C", [64, 32])
def test_converged_match_oracle(P, setup, C):
    inst, lp, dr, dc, eta, root, xr, yr, D = setup
    with make_ctx(inst, eta, scaling=1, eval_every=C) as ctx:
        ctx.set_batch(D, x_warm=xr, y_warm=yr, w_warm=np.full(len(D), root.w))
        ctx.solve(tol=1e-4, max_iters=50000)
        got = ctx.get_batch()
    for j, d in enumerate(D):
        r, x, y = S.solve_scaled(lp_for(lp, d), O.Options(tol=1e-4, max_iters=50000,
                                                          step_size=eta, eval_every=C),
                                 dr, dc, x_init=xr, y_init=yr, w_init=root.w)
        assert got["status"][j] == r.status and got["iters"][j] == r.iters, j
        assert rel_err(got["X"][j], x) <= 1e-8, j
        assert elem_err(got["X"][j], x) <= 1e-8, j
        assert got["obj"][j] == pytest.approx(r.obj, rel=1e-9, abs=1e-9)


def test_scaling_helps_the_badly_scaled_lp(P, setup):
    inst = setup[0]
    its = {}
    for sc in (0, 1):
        with make_ctx(inst, scaling=sc) as ctx:
            ctx.set_batch(obbt_deltas(choose_vars(inst.n, 2, seed=1))[:1])
            ctx.solve(tol=1e-4, max_iters=20000)
            its[sc] = int(ctx.get(0)["iters"])
    assert its[1] < its[0]


def test_serving_with_scaling_matches_batch(P, setup):
    inst, lp, dr, dc, eta, root, xr, yr, D = setup
    with make_ctx(inst, eta, scaling=1) as ctx:
        ctx.set_batch(D, x_warm=xr, y_warm=yr, w_warm=np.full(len(D), root.w))
        ctx.solve(tol=1e-4, max_iters=50000)
        ref = ctx.get_batch()
    with make_ctx(inst, eta, scaling=1) as ctx:
        ctx.set_base_warm(xr, yr, root.w)
        ctx.serve_begin(32)
        ids = list(ctx.submit(D, P.WARM_BASE, 1e-4, 50000))
        got = {}
        for _ in range(10000):
            if len(got) == len(ids):
                break
            ctx.serve_launch()
            ctx.serve_wait()
            for i in ctx.poll():
                got[i] = ctx.result(i)
    for j, i in enumerate(ids):
        assert got[i]["iters"] == ref["iters"][j]
        np.testing.assert_array_equal(got[i]["x"], ref["X"][j])
        np.testing.assert_array_equal(got[i]["y"], ref["Y"][j])
