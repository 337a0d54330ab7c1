"""Explicit single-LP data for the reference solver.

The LP is the primal problem of eq:main_lp (Section 3, Problem formulation):

    min c'x   s.t.   l <= A x <= u,   xl <= x <= xu

with row bounds (l, u) and variable bounds (xl, xu); an equality row has
l_i = u_i and infinite entries are allowed on the open side.  Instances arrive
as (A, c, b, sense, var bounds) and per-LP changes ("deltas"); this module turns
them into the explicit vectors of one LP, independently of the GPU library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

# delta kinds (same meaning as in the batch specification)
BASE, SET_LO, SET_HI, OBJ_UNIT = 0, 1, 2, 3


@dataclass
class LP:
    A: sp.csr_matrix     # m x n
    c: np.ndarray        # n
    l: np.ndarray        # m, row lower bounds (may be -inf)
    u: np.ndarray        # m, row upper bounds (may be +inf)
    xl: np.ndarray       # n, variable lower bounds (may be -inf)
    xu: np.ndarray       # n, variable upper bounds (may be +inf)
    b: np.ndarray        # m, right-hand side the rows came from (for the initial primal weight)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


def row_bounds(b: np.ndarray, sense: np.ndarray):
    """Map a right-hand side and row senses to the row interval [l, u] of eq:main_lp:
    'E' -> l = u = b;  'L' (Ax <= b) -> (-inf, b];  'G' (Ax >= b) -> [b, +inf);
    'N' -> a free row, (-inf, +inf)."""
    b = np.asarray(b, dtype=np.float64)
    s = np.asarray(sense)
    if s.dtype.kind in "SU":
        s = np.frombuffer("".join(s.astype(str)).encode(), dtype=np.uint8)
    l = np.empty_like(b)
    u = np.empty_like(b)
    for i in range(b.size):
        ch = chr(int(s[i]))
        if ch == "E":
            l[i], u[i] = b[i], b[i]
        elif ch == "L":
            l[i], u[i] = -np.inf, b[i]
        elif ch == "G":
            l[i], u[i] = b[i], np.inf
        elif ch == "N":
            l[i], u[i] = -np.inf, np.inf
        else:
            raise ValueError(f"unknown row sense {ch!r}")
    return l, u


def from_arrays(m, n, row_ptr, col_idx, val, c, b, sense, xl, xu) -> LP:
    A = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col_idx),
                       np.asarray(row_ptr)), shape=(m, n))
    l, u = row_bounds(b, sense)
    return LP(A=A, c=np.array(c, dtype=np.float64), l=l, u=u,
              xl=np.array(xl, dtype=np.float64), xu=np.array(xu, dtype=np.float64),
              b=np.array(b, dtype=np.float64))


def from_instance(inst) -> LP:
    """Base LP of a generated instance (any object with the CSR/vector fields)."""
    return from_arrays(inst.m, inst.n, inst.row_ptr, inst.col_idx, inst.val, inst.c,
                       inst.b, inst.sense, inst.l, inst.u)


def apply_delta(base: LP, kind: int, var: int, value: float) -> LP:
    """One member of a batch.  Strong branching changes one variable bound
    (Section 5.1: branch up raises xl_var, branch down lowers xu_var); bound
    tightening replaces the objective by value * e_var (Section 5.2).  All other
    data is shared with the base LP."""
    c, xl, xu = base.c, base.xl, base.xu
    if kind == BASE:
        pass
    elif kind == SET_LO:
        xl = xl.copy()
        xl[var] = value
    elif kind == SET_HI:
        xu = xu.copy()
        xu[var] = value
    elif kind == OBJ_UNIT:
        c = np.zeros(base.n)
        c[var] = value
    else:
        raise ValueError(f"unknown delta kind {kind}")
    return LP(A=base.A, c=c, l=base.l, u=base.u, xl=xl, xu=xu, b=base.b)
