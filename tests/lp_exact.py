"""Exact LP solutions for pinning the reference solver: brute-force vertex
enumeration on tiny LPs, the closed form of box-only LPs, and HiGHS (scipy)
with its duals mapped to the paper's sign convention."""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog


def vertex_enum(A: np.ndarray, l: np.ndarray, u: np.ndarray, xl: np.ndarray, xu: np.ndarray,
                c: np.ndarray, tol: float = 1e-9):
    """Minimum of c'x over {l <= Ax <= u, xl <= x <= xu} (finite box) by trying
    every choice of n linearly independent active hyperplanes."""
    m, n = A.shape
    planes = []   # (normal, rhs)
    for i in range(m):
        for bnd in {l[i], u[i]}:
            if np.isfinite(bnd):
                planes.append((A[i], bnd))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        planes.append((e, xl[j]))
        planes.append((e, xu[j]))
    best, best_x = np.inf, None
    for idx in itertools.combinations(range(len(planes)), n):
        M = np.array([planes[i][0] for i in idx])
        if abs(np.linalg.det(M)) < 1e-10:
            continue
        x = np.linalg.solve(M, np.array([planes[i][1] for i in idx]))
        ax = A @ x
        if np.all(x >= xl - tol) and np.all(x <= xu + tol) and np.all(ax >= l - tol) \
                and np.all(ax <= u + tol):
            v = c @ x
            if v < best:
                best, best_x = v, x
    return best, best_x


def box_closed_form(c: np.ndarray, xl: np.ndarray, xu: np.ndarray):
    """min c'x over a box: each x_j at the bound its cost sign selects."""
    x = np.where(c > 0, xl, np.where(c < 0, xu, np.clip(0.0, xl, xu)))
    return float(c @ x), x


def highs(lp):
    """Solve an oracle LP with HiGHS; return (obj, x, y) where y follows the
    paper's convention (y >= 0 on <= rows, y <= 0 on >= rows): the objective
    falls by y_i per unit increase of the active row bound."""
    A = lp.A
    eq = np.isfinite(lp.l) & np.isfinite(lp.u) & (lp.l == lp.u)
    le = ~eq & np.isfinite(lp.u)
    ge = ~eq & np.isfinite(lp.l)
    ile, ige, ieq = np.nonzero(le)[0], np.nonzero(ge)[0], np.nonzero(eq)[0]
    A_ub = sp.vstack([A[ile], -A[ige]]).tocsr()
    b_ub = np.concatenate([lp.u[ile], -lp.l[ige]])
    kw = {}
    if A_ub.shape[0]:
        kw.update(A_ub=A_ub, b_ub=b_ub)
    if ieq.size:
        kw.update(A_eq=A[ieq], b_eq=lp.u[ieq])
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b)
              for a, b in zip(lp.xl, lp.xu)]
    res = linprog(lp.c, bounds=bounds, method="highs", **kw)
    assert res.status == 0, res.message
    y = np.zeros(lp.m)
    if A_ub.shape[0]:
        mu = res.ineqlin.marginals        # d obj / d b_ub  (<= 0)
        y[ile] = -mu[: ile.size]
        y[ige] = mu[ile.size:]            # row -A x <= -l: d obj/d l = -mu, y = -d obj/d l
    if ieq.size:
        y[ieq] = -res.eqlin.marginals
    return float(res.fun), res.x, y
