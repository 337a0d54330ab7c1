"""MIP-facing outputs of a batch -- TEST INFRASTRUCTURE ONLY.

Turns the per-LP results of a strong-branching batch (Section 5.1) or a
bound-tightening batch (Section 5.2) into what a MIP solver consumes:
branching scores, and safe tightened variable bounds as in the OBBT
experiments of Section 6.  Plain FP64 scalar code; shares nothing with the GPU
library.

Readings (the paper leaves these open):
  * A bound is taken only from an LP that stopped optimal; an LP that hit its
    iteration limit or a numerical error gives none.  A primal-infeasible
    bound-tightening LP means the shared feasible set is empty.
  * OBBT: the bound computed for min x_v is the dual objective
    -phi_box(r) - phi_[l,u](y) at the returned point (weak duality makes it a
    lower bound); for max x_v, solved as min -x_v, it is minus that LP's dual
    objective.  The shift Delta uses the same LP's c'x and support values.
  * The improvement threshold is absolute: a bound moves only if the new value
    is better than the current one by more than the threshold.
  * Branching score: the gains are the child LPs' objective values c'x minus
    the parent's, floored at 0 (a restriction cannot lower the optimum; a
    negative value is solve error), +inf for an infeasible child (detected,
    or a branch whose new bound crosses the other bound).  The score
    combines them as (1 - mu) min + mu max with mu = 1/6, the weighting of the
    cited strong-branching study.

Pins: the bounds against exact variable ranges (vertex enumeration, HiGHS),
the gains against child optima.  Parity unpinned: the value mu = 1/6 (the
paper only says the children's objectives determine the score); the tests
pin the form of the score (a weighted mean of the smaller and the larger
gain), not the weight.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from .pdhg import Result, OPTIMAL, PRIMAL_INFEASIBLE, INFEASIBLE_BOUNDS

OBBT_DUAL_TOL = 1e-8        # dual-feasibility epsilon of the OBBT solves (Section 6)
OBBT_MIN_IMPROVE = 1e-4     # smallest bound change that is applied (Section 6)
SCORE_MU = 1.0 / 6.0


def safe_shift(eps: float, obj: float, dual_obj: float) -> float:
    """Delta = eps (1 + |c'x| + |phi_box(r) + phi_[l,u](y)|) (Section 6, OBBT
    results); phi_box(r) + phi_[l,u](y) is minus the dual objective."""
    return eps * (1.0 + abs(obj) + abs(dual_obj))


def obbt_bound(res: Result, sign: float, eps: float) -> Optional[float]:
    """Safe bound on x_v from the LP min sign * x_v (sign = +1 or -1, the
    objective e_v or -e_v of Section 5.2): weak duality gives
    sign * x_v >= D, so (D - Delta) / sign is a lower bound for sign = +1 and
    an upper bound (-D + Delta) for sign = -1; None when the LP gives none."""
    if res.status != OPTIMAL or res.kkt is None:
        return None
    d = res.kkt.dual_obj
    if not math.isfinite(d):
        return None
    delta = safe_shift(eps, res.kkt.obj, d)
    return (d - delta) / sign


@dataclass
class Tightened:
    xl: np.ndarray
    xu: np.ndarray
    changed: int            # bounds moved
    infeasible: bool        # some LP proved the feasible set empty


def obbt_tighten(xl, xu, var: Sequence[int], sign: Sequence[float], results: Sequence[Result],
                 eps: float = OBBT_DUAL_TOL, min_improve: float = OBBT_MIN_IMPROVE) -> Tightened:
    """x̲_v = max(x̲_v, lower OBBT bound), x̄_v = min(x̄_v, upper OBBT bound)
    (Section 5.2), with the safe shift and the improvement threshold of the OBBT
    experiments.  LP j minimised sign[j] * x_var[j]."""
    lo = np.array(xl, dtype=np.float64)
    hi = np.array(xu, dtype=np.float64)
    changed = 0
    infeasible = False
    for v, s, r in zip(var, sign, results):
        if r.status == PRIMAL_INFEASIBLE:
            infeasible = True
            continue
        b = obbt_bound(r, s, eps)
        if b is None:
            continue
        if s > 0 and b > lo[v] + min_improve:
            lo[v] = b
            changed += 1
        elif s < 0 and b < hi[v] - min_improve:
            hi[v] = b
            changed += 1
    return Tightened(lo, hi, changed, infeasible)


def branch_gain(child: Result, parent_obj: float) -> float:
    """Objective increase of a child LP over its parent (reading above)."""
    if child.status in (PRIMAL_INFEASIBLE, INFEASIBLE_BOUNDS):
        return math.inf
    if child.status != OPTIMAL:
        return math.nan
    return max(child.obj - parent_obj, 0.0)


def branch_score(gain_down: float, gain_up: float, mu: float = SCORE_MU) -> float:
    """(1 - mu) min(q-, q+) + mu max(q-, q+); NaN if either gain is unknown."""
    if math.isnan(gain_down) or math.isnan(gain_up):
        return math.nan
    lo, hi = min(gain_down, gain_up), max(gain_down, gain_up)
    if math.isinf(hi):
        return math.inf
    return (1.0 - mu) * lo + mu * hi
