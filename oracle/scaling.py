"""Diagonal preconditioning of the LP -- TEST INFRASTRUCTURE ONLY.

The paper names problem scaling among the enhancements of the first-order LP
method it builds on (Section 2) without making it part of its batched method;
this module adds it in front of the same solver.  With positive diagonal
matrices D_r (rows) and D_c (columns) the LP of eq:main_lp becomes

    min (D_c c)'x^  s.t.  D_r l <= (D_r A D_c) x^ <= D_r u,  D_c^-1 xl <= x^ <= D_c^-1 xu,

whose points map back as x = D_c x^ and y = D_r y^ (and r = D_c^-1 r^), with
equal primal and dual objectives.  The scaling itself follows the usual recipe
of that method: a few Ruiz equilibration passes (rows and columns divided by
the square roots of their infinity norms), then one Pock-Chambolle pass with
alpha = 1 (rows and columns divided by the square roots of their 1-norms).
Rows or columns without nonzeros keep the factor 1.

Reading: the stopping and infeasibility tests run on the scaled LP; the
tolerance refers to it.
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np
import scipy.sparse as sp

from .lp import LP, SET_LO, SET_HI, OBJ_UNIT
from .pdhg import Options, Result, solve

RUIZ_ITERS = 10
PC_ALPHA = 1.0


def _row_inf(A: sp.csr_matrix) -> np.ndarray:
    return np.asarray(abs(A).max(axis=1).todense()).ravel()


def _col_inf(A: sp.csr_matrix) -> np.ndarray:
    return np.asarray(abs(A).max(axis=0).todense()).ravel()


def _safe_inv_sqrt(v: np.ndarray) -> np.ndarray:
    out = np.ones_like(v)
    nz = v > 0.0
    out[nz] = 1.0 / np.sqrt(v[nz])
    return out


def scaled_matrix(A: sp.csr_matrix, dr: np.ndarray, dc: np.ndarray) -> sp.csr_matrix:
    """D_r A D_c."""
    return sp.csr_matrix(sp.diags(dr) @ A @ sp.diags(dc))


def ruiz(A: sp.csr_matrix, iters: int = RUIZ_ITERS) -> Tuple[np.ndarray, np.ndarray]:
    """Ruiz equilibration: each pass divides every row and column of the
    current scaled matrix by the square root of its infinity norm."""
    m, n = A.shape
    dr, dc = np.ones(m), np.ones(n)
    for _ in range(iters):
        S = scaled_matrix(A, dr, dc)
        dr = dr * _safe_inv_sqrt(_row_inf(S))
        dc = dc * _safe_inv_sqrt(_col_inf(S))
    return dr, dc


def pock_chambolle(A: sp.csr_matrix, dr: np.ndarray, dc: np.ndarray,
                   alpha: float = PC_ALPHA) -> Tuple[np.ndarray, np.ndarray]:
    """One Pock-Chambolle pass on D_r A D_c: rows divided by
    sqrt(sum_j |a_ij|^(2 - alpha)), columns by sqrt(sum_i |a_ij|^alpha)."""
    S = abs(scaled_matrix(A, dr, dc))
    rows = np.asarray(S.power(2.0 - alpha).sum(axis=1)).ravel()
    cols = np.asarray(S.power(alpha).sum(axis=0)).ravel()
    return dr * _safe_inv_sqrt(rows), dc * _safe_inv_sqrt(cols)


def scaling(A: sp.csr_matrix, ruiz_iters: int = RUIZ_ITERS,
            alpha: Optional[float] = PC_ALPHA) -> Tuple[np.ndarray, np.ndarray]:
    dr, dc = ruiz(A, ruiz_iters)
    if alpha is not None:
        dr, dc = pock_chambolle(A, dr, dc, alpha)
    return dr, dc


def scale_lp(lp: LP, dr: np.ndarray, dc: np.ndarray) -> LP:
    """The scaled LP (module docstring).  Infinite bounds stay infinite."""
    with np.errstate(invalid="ignore"):
        return LP(A=scaled_matrix(lp.A, dr, dc), c=dc * lp.c, l=dr * lp.l, u=dr * lp.u,
                  xl=lp.xl / dc, xu=lp.xu / dc, b=dr * lp.b)


def scale_delta(kind: int, var: int, value: float, dc: np.ndarray) -> float:
    """A change of the original LP expressed on the scaled one: a bound on x_var
    becomes value / dc[var]; the objective value * e_var becomes
    value * dc[var] * e_var."""
    if kind in (SET_LO, SET_HI):
        return value / dc[var]
    if kind == OBJ_UNIT:
        return value * dc[var]
    return value


def unscale(x_hat: np.ndarray, y_hat: np.ndarray, dr: np.ndarray,
            dc: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    return dc * x_hat, dr * y_hat


def solve_scaled(lp: LP, opt: Options, dr: np.ndarray, dc: np.ndarray,
                 x_init=None, y_init=None, w_init=None) -> Tuple[Result, np.ndarray, np.ndarray]:
    """Solve the scaled LP from a start given in original coordinates; return
    the result on the scaled LP and its point mapped back (x, y)."""
    s = scale_lp(lp, dr, dc)
    xi = None if x_init is None else np.asarray(x_init) / dc
    yi = None if y_init is None else np.asarray(y_init) / dr
    res = solve(s, opt, x_init=xi, y_init=yi, w_init=w_init)
    x, y = unscale(res.x, res.y, dr, dc)
    return res, x, y
