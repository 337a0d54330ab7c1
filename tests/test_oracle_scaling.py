"""Pins for the diagonal preconditioning: closed forms (a diagonal matrix is
equilibrated in one pass), the Pock-Chambolle bound ||D_r A D_c||_2 <= 1, the
convergence of Ruiz passes, the invariance of both objectives and of the gap
under scaling, the mapping of per-LP changes, and optima of tiny LPs solved
scaled against vertex enumeration."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle import scaling as S
from tests.lp_exact import vertex_enum
from workloads import make_tiny, make_cfg1


def _wild(seed, m=30, n=50, density=0.15):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=density, random_state=rng, format="csr")
    A.data = rng.choice([-1.0, 1.0], A.nnz) * 10.0 ** rng.uniform(-3, 3, A.nnz)
    return A


def test_diagonal_matrix_equilibrated_in_one_pass():
    a = np.array([2.0, -8.0, 0.5, 1e-3])
    A = sp.csr_matrix(np.diag(a))
    dr, dc = S.ruiz(A, iters=1)
    np.testing.assert_allclose(S.scaled_matrix(A, dr, dc).toarray(), np.diag(np.sign(a)),
                               rtol=1e-15)
    dr10, dc10 = S.ruiz(A, iters=10)
    np.testing.assert_allclose(dr10, dr, rtol=1e-15)
    np.testing.assert_allclose(dc10, dc, rtol=1e-15)


def test_empty_rows_and_columns_keep_factor_one():
    A = sp.csr_matrix(np.array([[0.0, 0.0, 0.0], [0.0, 4.0, 0.0]]))
    dr, dc = S.scaling(A)
    assert dr[0] == 1.0 and dc[0] == 1.0 and dc[2] == 1.0


@pytest.mark.parametrize("seed", range(3))
def test_ruiz_equilibrates(seed):
    A = _wild(seed)
    dr, dc = S.ruiz(A, iters=10)
    Sm = abs(S.scaled_matrix(A, dr, dc))
    r = np.asarray(Sm.max(axis=1).todense()).ravel()
    c = np.asarray(Sm.max(axis=0).todense()).ravel()
    assert np.max(np.abs(np.log(r[r > 0]))) < 0.02
    assert np.max(np.abs(np.log(c[c > 0]))) < 0.02


@pytest.mark.parametrize("seed", range(3))
def test_pock_chambolle_bounds_the_norm(seed):
    A = _wild(seed)
    for dr0, dc0 in ((np.ones(A.shape[0]), np.ones(A.shape[1])), S.ruiz(A)):
        dr, dc = S.pock_chambolle(A, dr0, dc0, alpha=1.0)
        assert O.opnorm(S.scaled_matrix(A, dr, dc)) <= 1.0 + 1e-9
        # the raw matrix's norm is far above 1
    assert O.opnorm(A) > 10.0


@pytest.mark.parametrize("seed", range(4))
def test_objectives_and_gap_invariant(seed):
    lp = O.from_instance(make_tiny(seed, m=4, n=6, senses="ELG", box=(0.0, 4.0)))
    dr, dc = S.scaling(lp.A)
    s = S.scale_lp(lp, dr, dc)
    rng = np.random.default_rng(seed)
    for _ in range(5):
        xh = rng.uniform(-1, 5, lp.n)
        yh = rng.normal(size=lp.m)
        yh = O.proj_barrier_cone(yh, s.l, s.u)
        x, y = S.unscale(xh, yh, dr, dc)
        ks, ko = O.kkt(s, xh, yh), O.kkt(lp, x, y)
        assert ks.obj == pytest.approx(ko.obj, rel=1e-12, abs=1e-12)
        assert ks.dual_obj == pytest.approx(ko.dual_obj, rel=1e-10, abs=1e-10)
        assert ks.gap == pytest.approx(ko.gap, rel=1e-9, abs=1e-12)


def test_delta_mapping_commutes():
    lp = O.from_instance(make_cfg1())
    dr, dc = S.scaling(lp.A)
    s = S.scale_lp(lp, dr, dc)
    for kind, var, val in ((O.SET_LO, 7, 6.0), (O.SET_HI, 11, 2.0), (O.OBJ_UNIT, 3, -1.0)):
        a = S.scale_lp(O.apply_delta(lp, kind, var, val), dr, dc)
        b = O.apply_delta(s, kind, var, S.scale_delta(kind, var, val, dc))
        np.testing.assert_allclose(a.c, b.c, rtol=1e-15)
        np.testing.assert_allclose(a.xl, b.xl, rtol=1e-15)
        np.testing.assert_allclose(a.xu, b.xu, rtol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_scaled_solve_reaches_the_exact_optimum(seed):
    inst = make_tiny(seed, m=3, n=5, senses="ELG", box=(0.0, 4.0))
    lp = O.from_instance(inst)
    exact, _ = vertex_enum(lp.A.toarray(), lp.l, lp.u, lp.xl, lp.xu, lp.c)
    dr, dc = S.scaling(lp.A)
    res, x, y = S.solve_scaled(lp, O.Options(tol=1e-9, max_iters=400000), dr, dc)
    assert res.status == O.OPTIMAL
    assert lp.c @ x == pytest.approx(exact, abs=1e-6 * (1 + abs(exact)))
    assert np.all(x >= lp.xl - 1e-9) and np.all(x <= lp.xu + 1e-9)
    assert O.kkt(lp, x, y).rel <= 1e-6
