"""Reference restarted, reflected-Halpern PDHG for one LP at a time (FP64).

Plain numpy/scipy, written from the paper's Sections 3-5 (arXiv 2601.21990,
"Batched First-Order Methods for Parallel LP Solving in MIP").  No blocking,
fusion or reordering beyond the definitions: each function names the passage
it restates.  Where the paper is silent or its printed formula conflicts with
the rest of the method, the reading taken is stated in the docstring and
selectable through ``Options``.

Test infrastructure only: the GPU library never imports, links or calls this.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from .lp import LP

# per-LP outcomes (statuses, not errors)
RUNNING = 0
OPTIMAL = 1
ITERATION_LIMIT = 2
INFEASIBLE_BOUNDS = 3
NUMERICAL_ERROR = 4
PRIMAL_INFEASIBLE = 6
DUAL_INFEASIBLE = 7

STATUS_NAMES = {RUNNING: "RUNNING", OPTIMAL: "OPTIMAL", ITERATION_LIMIT: "ITERATION_LIMIT",
                INFEASIBLE_BOUNDS: "INFEASIBLE_BOUNDS", NUMERICAL_ERROR: "NUMERICAL_ERROR",
                PRIMAL_INFEASIBLE: "PRIMAL_INFEASIBLE", DUAL_INFEASIBLE: "DUAL_INFEASIBLE"}


# ---------------------------------------------------------------------------
# elementary operators (Section 3 and Section 4)
# ---------------------------------------------------------------------------

def proj_box(v: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Euclidean projection onto the box [a, b]: max{min{v, b}, a} elementwise (Section 4)."""
    return np.maximum(np.minimum(v, b), a)


def support(v: np.ndarray, a: np.ndarray, b: np.ndarray) -> float:
    """Support function of the box [a, b]: sup over z in [a,b] of v'z = b'v_+ + a'v_-
    (Section 3).  A zero component contributes zero even against an infinite
    bound (0 * inf := 0); a component pointing at an infinite side gives +inf."""
    vp = np.maximum(v, 0.0)
    vm = np.minimum(v, 0.0)
    with np.errstate(invalid="ignore"):
        tp = np.where(vp > 0.0, b * vp, 0.0)
        tm = np.where(vm < 0.0, a * vm, 0.0)
    return float(np.sum(tp) + np.sum(tm))


def proj_barrier_cone(v: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Projection onto the barrier cone of [a, b] (Section 3):
    B = {v : v_i >= 0 if a_i = -inf;  v_i <= 0 if b_i = +inf;  free otherwise}.
    A coordinate with both sides infinite must be >= 0 and <= 0, i.e. zero."""
    out = np.array(v, dtype=np.float64, copy=True)
    lo_inf = np.isneginf(a)
    hi_inf = np.isposinf(b)
    out[lo_inf] = np.maximum(out[lo_inf], 0.0)
    out[hi_inf] = np.minimum(out[hi_inf], 0.0)
    return out


def proj_recession_cone(v: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Projection onto the recession cone of the box [a, b] (Section 4, infeasibility
    detection).  The printed definition lists v_i >= 0 when b_i = +inf and v_i <= 0
    when the lower end is -inf, 0 otherwise, which contradicts itself for a free
    coordinate.  Reading: free coordinate (both ends infinite) -> unconstrained;
    only b_i = +inf -> v_i >= 0; only a_i = -inf -> v_i <= 0; both finite -> 0."""
    out = np.array(v, dtype=np.float64, copy=True)
    lo_inf = np.isneginf(a)
    hi_inf = np.isposinf(b)
    out[~lo_inf & ~hi_inf] = 0.0
    up = hi_inf & ~lo_inf
    dn = lo_inf & ~hi_inf
    out[up] = np.maximum(out[up], 0.0)
    out[dn] = np.minimum(out[dn], 0.0)
    return out


def pdhg_operator(lp: LP, x: np.ndarray, y: np.ndarray, tau: float, sigma: float):
    """The PDHG operator T of Section 4 for the saddle problem eq:lp_saddle:
        x~ = Pi_[xl,xu]( x - tau (c + A'y) )
        y~ = y + sigma A(2x~ - x) - sigma Pi_[l,u]( y/sigma + A(2x~ - x) ).
    The dual line is evaluated as y~ = sigma (q - Pi_[l,u](q)) with
    q = y/sigma + A(2x~ - x), which is the same expression in exact arithmetic.
    In floating point the printed order leaves rounding residue of either sign
    where the projection is inactive (q strictly inside [l, u]), which puts y~
    outside the barrier cone of a one-sided row and makes phi_[l,u](y~)
    infinite; this order returns exactly zero there.
    """
    x_t = proj_box(x - tau * (lp.c + lp.A.T @ y), lp.xl, lp.xu)
    v = lp.A @ (2.0 * x_t - x)
    q = y / sigma + v
    y_t = sigma * (q - proj_box(q, lp.l, lp.u))
    return x_t, y_t


def fixed_point_residual(lp: LP, x, y, x_t, y_t, w: float, eta: float,
                         cross_sign: float = -1.0) -> float:
    """r(z) = ||T(z) - z||_M of eq:residual with
        M = [[ (w/eta) I, s A' ], [ s A, 1/(eta w) I ]].
    The paper prints s = +1; with its own sign convention for T (+A'y in the
    primal step, +A(2x~-x) in the dual step) the metric in which T is firmly
    nonexpansive has s = -1, which is the default reading (cross_sign)."""
    dx = x_t - x
    dy = y_t - y
    q = (w / eta) * float(dx @ dx) + (1.0 / (eta * w)) * float(dy @ dy) \
        + 2.0 * cross_sign * float(dy @ (lp.A @ dx))
    if not np.isfinite(q):
        return float("nan")
    return math.sqrt(max(q, 0.0))


@dataclass
class KKT:
    gap: float
    primal: float
    dual: float
    rel: float          # max of the three relative measures
    obj: float          # c'x
    dual_obj: float     # -phi_box(r) - phi_[l,u](y)


def reduced_cost(lp: LP, y: np.ndarray) -> np.ndarray:
    """r = Pi_B[xl,xu]( -c - A'y ) (Section 4, stopping criteria)."""
    return proj_barrier_cone(-lp.c - lp.A.T @ y, lp.xl, lp.xu)


def kkt(lp: LP, x: np.ndarray, y: np.ndarray) -> KKT:
    """Relative optimality measures of eq:stopping at (x, y):
        gap    = |c'x + phi_box(r) + phi_[l,u](y)| / (1 + |c'x| + |phi_box(r) + phi_[l,u](y)|)
        primal = ||Ax - Pi_[l,u](Ax)|| / (1 + ||Ax||)
        dual   = ||c + A'y + r|| / (1 + ||c||)
    eq:stopping states three separate tests against one epsilon; they hold
    together iff their maximum is <= epsilon, which is what `rel` reports."""
    r = reduced_cost(lp, y)
    cx = float(lp.c @ x)
    phis = support(r, lp.xl, lp.xu) + support(y, lp.l, lp.u)
    if np.isfinite(phis):
        gap = abs(cx + phis) / (1.0 + abs(cx) + abs(phis))
    else:
        gap = float("inf")
    ax = lp.A @ x
    primal = float(np.linalg.norm(ax - proj_box(ax, lp.l, lp.u))) / (1.0 + float(np.linalg.norm(ax)))
    dual = float(np.linalg.norm(lp.c + lp.A.T @ y + r)) / (1.0 + float(np.linalg.norm(lp.c)))
    rel = max(gap, primal, dual)
    if any(math.isnan(v) for v in (gap, primal, dual)):
        rel = float("nan")
    return KKT(gap=gap, primal=primal, dual=dual, rel=rel, obj=cx, dual_obj=-phis)


@dataclass
class Infeasibility:
    primal: bool
    dual: bool
    primal_ratio: float     # ||A'dy + dr|| / |phi(dy) + phi(dr)|   (inf when phi >= 0)
    dual_ratio: float       # max of the two recession residuals / |c'dx|  (inf when c'dx >= 0)


def infeasibility(lp: LP, x, y, x_t, y_t, eps: float) -> Infeasibility:
    """eps-approximate infeasibility tests of Section 4 (eq:primal-infeas,
    eq:dual-infeas) on the displacement of one application of T:
        dx = x~ - x,  dy = Pi_B[l,u](y~ - y),  dr = Pi_B[xl,xu](r~ - r),
    r = Pi_B[xl,xu](-c - A'y), r~ = Pi_B[xl,xu](-c - A'y~).
      primal infeasible:  phi_[l,u](dy) + phi_box(dr) < 0  and
                          ||A'dy + dr|| <= eps |phi_[l,u](dy) + phi_box(dr)|
      dual infeasible:    c'dx < 0,  ||dx - Pi_R[xl,xu](dx)|| <= eps |c'dx|,
                          ||A dx - Pi_R[l,u](A dx)|| <= eps |c'dx|.
    The printed right-hand side of the second primal test, eps(phi(dy) + phi(dr)),
    is negative whenever the first test holds; reading: its absolute value."""
    r = reduced_cost(lp, y)
    r_t = reduced_cost(lp, y_t)
    dx = x_t - x
    dy = proj_barrier_cone(y_t - y, lp.l, lp.u)
    dr = proj_barrier_cone(r_t - r, lp.xl, lp.xu)
    phi = support(dy, lp.l, lp.u) + support(dr, lp.xl, lp.xu)
    if phi < 0.0:
        pr = float(np.linalg.norm(lp.A.T @ dy + dr)) / abs(phi)
    else:
        pr = float("inf")
    cdx = float(lp.c @ dx)
    if cdx < 0.0:
        adx = lp.A @ dx
        res = max(float(np.linalg.norm(dx - proj_recession_cone(dx, lp.xl, lp.xu))),
                  float(np.linalg.norm(adx - proj_recession_cone(adx, lp.l, lp.u))))
        dr_ = res / abs(cdx)
    else:
        dr_ = float("inf")
    return Infeasibility(primal=pr <= eps, dual=dr_ <= eps, primal_ratio=pr, dual_ratio=dr_)


# ---------------------------------------------------------------------------
# step size, primal weight, restart rule (Section 4)
# ---------------------------------------------------------------------------

def opnorm(A, tol: float = 1e-14, maxit: int = 10000) -> float:
    """Spectral norm ||A||_2 for the constant step size.  The paper does not say
    how it is computed; this is power iteration on A'A, stopped when the
    eigenvalue estimate changes by at most `tol` relative (or after `maxit`
    products).  The start vector is v_j = 1 + frac(j g), g = (sqrt(5)-1)/2 (a
    Weyl sequence), normalised: a constant start vector lies in the null space
    of matrices whose rows sum to zero (e.g. A = [1, -1])."""
    n = A.shape[1]
    if n == 0 or A.nnz == 0:
        return 0.0
    v = 1.0 + np.modf(np.arange(n, dtype=np.float64) * 0.6180339887498949)[0]
    v = v / np.linalg.norm(v)
    lam_old = 0.0
    lam = 0.0
    for _ in range(maxit):
        w = A.T @ (A @ v)
        lam = float(np.linalg.norm(w))
        if lam == 0.0:
            return 0.0
        v = w / lam
        if abs(lam - lam_old) <= tol * lam:
            break
        lam_old = lam
    return math.sqrt(lam)


def step_size(A) -> float:
    """eta = 0.998 / ||A||_2 (Section 4, step-size and primal weight); eta = 1 if A = 0."""
    s = opnorm(A)
    return 0.998 / s if s > 0.0 else 1.0


def initial_primal_weight(lp: LP) -> float:
    """Not stated in the paper.  Reading: ||c|| / ||b|| when both exceed 1e-10, else 1."""
    nc = float(np.linalg.norm(lp.c))
    nb = float(np.linalg.norm(lp.b))
    if nc > 1e-10 and nb > 1e-10:
        return nc / nb
    return 1.0


def smoothed_primal_weight(dx_norm: float, dy_norm: float, w: float, theta: float,
                           ratio: str = "dy/dx") -> float:
    """w+ = exp(theta log d + (1 - theta) log w), applied only when d is finite
    (Section 4).  d is the ratio of the anchor displacements of consecutive
    restarts.  The paper prints d = ||dx|| / ||dy||; with tau = eta/w and
    sigma = eta w, balancing the two diagonal blocks of the residual metric
    gives d = ||dy|| / ||dx||, the default reading (`ratio`).  "Finite" is read
    as both norms above 1e-10."""
    num, den = (dy_norm, dx_norm) if ratio == "dy/dx" else (dx_norm, dy_norm)
    if num > 1e-10 and den > 1e-10 and math.isfinite(num) and math.isfinite(den):
        d = num / den
        return math.exp(theta * math.log(d) + (1.0 - theta) * math.log(w))
    return w


def restart_due(r: float, r0: float, r_prev: Optional[float], k: int, t: int,
                beta_s: float, beta_n: float, beta_a: float) -> bool:
    """The three restart conditions of Section 4 (Restarts):
      sufficient decay     r(z^{n,k}) <= beta_s r(z^{n,0});
      necessary decay and  r(z^{n,k}) <= beta_n r(z^{n,0}) and r(z^{n,k}) > r(z^{n,k-1});
        no inner progress
      iteration limit      k > beta_a K, K the total number of iterations so far.
    r(z^{n,k-1}) is the previous evaluated residual of this restart cycle."""
    if r <= beta_s * r0:
        return True
    if r_prev is not None and r <= beta_n * r0 and r > r_prev:
        return True
    if k > beta_a * t:
        return True
    return False


# ---------------------------------------------------------------------------
# the solver
# ---------------------------------------------------------------------------

@dataclass
class Options:
    tol: float = 1e-4
    max_iters: int = 100000
    eval_every: int = 64            # C: KKT and restart tests at t mod C == 0
    beta_s: float = 0.2
    beta_n: float = 0.8
    beta_a: float = 0.36
    theta: float = 0.5
    step_size: Optional[float] = None    # eta; None -> 0.998/||A||_2
    cross_sign: float = -1.0
    pw_ratio: str = "dy/dx"
    infeas_tol: Optional[float] = None   # eps of the infeasibility tests; None: tol; 0: off
    dual_tol: Optional[float] = None     # eps of the dual-feasibility test; None: tol
    # S: stopping tests also at t mod S == 0 between the evaluations above
    # (0: off; S >= 2 dividing C; per-LP restart scope only)
    stop_every: int = 0


@dataclass
class Result:
    status: int
    x: np.ndarray                   # x~ at termination (the returned primal point)
    y: np.ndarray                   # y~ at termination
    x_iter: Optional[np.ndarray]    # Halpern iterate after the last update
    y_iter: Optional[np.ndarray]
    iters: int                      # applications of T
    restarts: List[int] = field(default_factory=list)   # iteration indices t of restarts
    w: float = float("nan")
    eta: float = float("nan")
    kkt: Optional[KKT] = None

    @property
    def obj(self) -> float:
        return self.kkt.obj if self.kkt is not None else float("nan")


def _stop_every(opt: "Options") -> int:
    """The interval S of the extra stopping tests, 0 when off; S must be at
    least 2 and divide C (so they never fall on t = 0 mod C or on the first
    iteration of a restart cycle)."""
    S = int(opt.stop_every)
    if S == 0 or S == opt.eval_every:
        return 0
    if S < 2 or opt.eval_every % S != 0:
        raise ValueError("stop_every must be 0 or a divisor >= 2 of eval_every")
    return S


def _converged(kk: KKT, opt: "Options") -> bool:
    """eq:stopping with one epsilon for the gap and primal tests and another
    for the dual-feasibility test.  The bound-tightening experiments (Section 6,
    OBBT results) check dual feasibility more strictly than the rest; by
    default the two are equal, and then this is max(gap, primal, dual) <= tol."""
    eps_d = opt.tol if opt.dual_tol is None else opt.dual_tol
    return kk.gap <= opt.tol and kk.primal <= opt.tol and kk.dual <= eps_d


def _infeasibility_eps(opt: "Options") -> float:
    """The infeasibility tests of Section 4 are stated with the same epsilon as
    the stopping criteria (eq:stopping) and no separate value is given; reading:
    the stopping tolerance unless an explicit value is set."""
    return opt.tol if opt.infeas_tol is None else opt.infeas_tol


def _infeasible_status(inf: Infeasibility) -> int:
    """Primal infeasibility is reported first when both tests pass."""
    if inf.primal:
        return PRIMAL_INFEASIBLE
    if inf.dual:
        return DUAL_INFEASIBLE
    return 0


def _halpern(k: int, x_t, x, x_anchor):
    """Reflected Halpern step of eq:mainiter:
       z^{k+1} = (k+1)/(k+2) (2 T(z^k) - z^k) + 1/(k+2) z^0."""
    return (k + 1) / (k + 2) * (2.0 * x_t - x) + x_anchor / (k + 2)


def solve(lp: LP, opt: Options = Options(), x_init=None, y_init=None,
          w_init: Optional[float] = None) -> Result:
    """Restarted reflected-Halpern PDHG on one LP (Section 4).

    Schedule (the paper leaves it open; reading shared with the GPU library):
      * t counts applications of T from 0, k counts them inside a restart cycle;
      * the residual r is evaluated when k == 0 (it becomes r(z^{n,0})) and at
        every t with t mod C == 0, where also the stopping test runs at
        z~ = T(z^t) and the restart conditions are tested (k > 0);
      * on restart the anchor and the iterate both become z~, the primal weight
        is smoothed from the anchor displacement, k returns to 0 and the
        iteration counts as spent;
      * the LP stops OPTIMAL when max(gap, primal, dual) <= tol at an evaluation
        point, PRIMAL_INFEASIBLE / DUAL_INFEASIBLE when the infeasibility tests
        pass there (after the stopping test), and ITERATION_LIMIT after
        max_iters applications of T; in every case it returns z~ of its last
        iteration;
      * with stop_every = S, the stopping test (eq:stopping at z~, and the NaN
        check) also runs at every t with t mod S == 0 between those evaluation
        points; nothing else happens there (no residual, no restart or
        infeasibility test), so the iterates are those of the run without it
        and the LP only stops sooner.
    """
    n, m = lp.n, lp.m
    if np.any(lp.xl > lp.xu):
        z = np.zeros(n)
        return Result(status=INFEASIBLE_BOUNDS, x=z, y=np.zeros(m), x_iter=None, y_iter=None,
                      iters=0)
    eta = opt.step_size if opt.step_size is not None else step_size(lp.A)
    w = float(w_init) if w_init is not None else initial_primal_weight(lp)
    x = proj_box(np.zeros(n) if x_init is None else np.asarray(x_init, dtype=np.float64),
                 lp.xl, lp.xu)
    y = np.zeros(m) if y_init is None else np.array(y_init, dtype=np.float64)
    x_a, y_a = x, y
    k = 0
    t = 0
    r0 = None
    r_prev = None
    restarts: List[int] = []
    C = opt.eval_every
    S = _stop_every(opt)
    eps_inf = _infeasibility_eps(opt)

    while True:
        tau, sigma = eta / w, eta * w
        x_t, y_t = pdhg_operator(lp, x, y, tau, sigma)
        full = (t % C == 0)
        evaluate = full or k == 0
        r = fixed_point_residual(lp, x, y, x_t, y_t, w, eta, opt.cross_sign) if evaluate else None
        kk = None
        if full or (S and t % S == 0):
            kk = kkt(lp, x_t, y_t)
        if (r is not None and not math.isfinite(r)) or (kk is not None and not math.isfinite(kk.rel)):
            return Result(NUMERICAL_ERROR, x_t, y_t, None, None, t + 1, restarts, w, eta,
                          kk or kkt(lp, x_t, y_t))
        if kk is not None and _converged(kk, opt):
            return Result(OPTIMAL, x_t, y_t, _halpern(k, x_t, x, x_a), _halpern(k, y_t, y, y_a),
                          t + 1, restarts, w, eta, kk)
        if full and eps_inf > 0.0:
            st = _infeasible_status(infeasibility(lp, x, y, x_t, y_t, eps_inf))
            if st:
                return Result(st, x_t, y_t, _halpern(k, x_t, x, x_a), _halpern(k, y_t, y, y_a),
                              t + 1, restarts, w, eta, kk)
        if t + 1 >= opt.max_iters:
            return Result(ITERATION_LIMIT, x_t, y_t, _halpern(k, x_t, x, x_a),
                          _halpern(k, y_t, y, y_a), t + 1, restarts, w, eta,
                          kk or kkt(lp, x_t, y_t))
        if k == 0:
            r0 = r
        elif full and restart_due(r, r0, r_prev, k, t, opt.beta_s, opt.beta_n, opt.beta_a):
            w = smoothed_primal_weight(float(np.linalg.norm(x_t - x_a)),
                                       float(np.linalg.norm(y_t - y_a)), w, opt.theta,
                                       opt.pw_ratio)
            x, y = x_t, y_t
            x_a, y_a = x_t, y_t
            restarts.append(t)
            k = 0
            t += 1
            r_prev = None
            continue
        if evaluate:
            r_prev = r
        x, y = _halpern(k, x_t, x, x_a), _halpern(k, y_t, y, y_a)
        k += 1
        t += 1


def solve_batch_avg(lps: Sequence[LP], opt: Options = Options(), x_inits=None, y_inits=None,
                    w_inits=None) -> List[Result]:
    """Batched restart scope of Section 5 (Restarts): every LP runs the same
    iteration with its own primal weight and step sizes, the restart tests use
    the average residual over the batch, and when they fire all LPs restart
    together, each smoothing its own weight.  The paper does not say which LPs
    enter the average once some have stopped; reading: the LPs still running
    after this evaluation's stopping tests.  The extra stopping tests of
    stop_every belong to the per-LP scope only (an LP leaving between two
    evaluations would change the average the others restart on)."""
    if _stop_every(opt):
        raise ValueError("stop_every applies to the per-LP restart scope only")
    N = len(lps)
    res: List[Optional[Result]] = [None] * N
    state = []
    for j, lp in enumerate(lps):
        if np.any(lp.xl > lp.xu):
            res[j] = Result(INFEASIBLE_BOUNDS, np.zeros(lp.n), np.zeros(lp.m), None, None, 0)
            state.append(None)
            continue
        eta = opt.step_size if opt.step_size is not None else step_size(lp.A)
        w = float(w_inits[j]) if w_inits is not None else initial_primal_weight(lp)
        x = proj_box(np.zeros(lp.n) if x_inits is None else np.asarray(x_inits[j], dtype=np.float64),
                     lp.xl, lp.xu)
        y = np.zeros(lp.m) if y_inits is None else np.array(y_inits[j], dtype=np.float64)
        state.append(dict(eta=eta, w=w, x=x, y=y, xa=x, ya=y, restarts=[]))
    active = [j for j in range(N) if state[j] is not None]
    eps_inf = _infeasibility_eps(opt)
    k, t = 0, 0
    r0 = None
    r_prev = None
    C = opt.eval_every
    while active:
        full = (t % C == 0)
        evaluate = full or k == 0
        steps = {}
        for j in active:
            s = state[j]
            x_t, y_t = pdhg_operator(lps[j], s["x"], s["y"], s["eta"] / s["w"], s["eta"] * s["w"])
            r = (fixed_point_residual(lps[j], s["x"], s["y"], x_t, y_t, s["w"], s["eta"],
                                      opt.cross_sign) if evaluate else None)
            steps[j] = (x_t, y_t, r)
        still = []
        for j in active:
            s = state[j]
            x_t, y_t, r = steps[j]
            kk = kkt(lps[j], x_t, y_t) if full else None
            hx = lambda: _halpern(k, x_t, s["x"], s["xa"])
            hy = lambda: _halpern(k, y_t, s["y"], s["ya"])
            if (r is not None and not math.isfinite(r)) or (kk is not None and not math.isfinite(kk.rel)):
                res[j] = Result(NUMERICAL_ERROR, x_t, y_t, None, None, t + 1, s["restarts"], s["w"],
                                s["eta"], kk or kkt(lps[j], x_t, y_t))
            elif kk is not None and _converged(kk, opt):
                res[j] = Result(OPTIMAL, x_t, y_t, hx(), hy(), t + 1, s["restarts"], s["w"], s["eta"], kk)
            elif full and eps_inf > 0.0 and _infeasible_status(
                    infeasibility(lps[j], s["x"], s["y"], x_t, y_t, eps_inf)):
                st = _infeasible_status(infeasibility(lps[j], s["x"], s["y"], x_t, y_t, eps_inf))
                res[j] = Result(st, x_t, y_t, hx(), hy(), t + 1, s["restarts"], s["w"], s["eta"], kk)
            elif t + 1 >= opt.max_iters:
                res[j] = Result(ITERATION_LIMIT, x_t, y_t, hx(), hy(), t + 1, s["restarts"], s["w"],
                                s["eta"], kk or kkt(lps[j], x_t, y_t))
            else:
                still.append(j)
        active = still
        if not active:
            break
        r_bar = float(np.mean([steps[j][2] for j in active])) if evaluate else None
        if k == 0:
            r0 = r_bar
        elif full and restart_due(r_bar, r0, r_prev, k, t, opt.beta_s, opt.beta_n, opt.beta_a):
            for j in active:
                s = state[j]
                x_t, y_t, _ = steps[j]
                s["w"] = smoothed_primal_weight(float(np.linalg.norm(x_t - s["xa"])),
                                                float(np.linalg.norm(y_t - s["ya"])), s["w"],
                                                opt.theta, opt.pw_ratio)
                s["x"], s["y"], s["xa"], s["ya"] = x_t, y_t, x_t, y_t
                s["restarts"].append(t)
            k = 0
            t += 1
            r_prev = None
            continue
        if evaluate:
            r_prev = r_bar
        for j in active:
            s = state[j]
            x_t, y_t, _ = steps[j]
            s["x"], s["y"] = _halpern(k, x_t, s["x"], s["xa"]), _halpern(k, y_t, s["y"], s["ya"])
        k += 1
        t += 1
    return res  # type: ignore[return-value]
