"""FP64 reference solver for the batched PDHG library -- TEST INFRASTRUCTURE ONLY.

A plain, slow CPU implementation of what the GPU path computes, written from
arXiv 2601.21990 (Sections 3-5): the LP and its saddle form, the PDHG operator,
reflected Halpern iterations, the fixed-point residual, adaptive restarts,
primal-weight smoothing, the stopping criteria and the batched restart scope.
It solves one LP at a time in float64 with numpy/scipy.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library (kernels, headers,
helpers or constants), and the GPU library never calls it.

Also: `oracle.mip` (safe bound-tightening bounds and strong-branching scores
from per-LP results, Sections 5.1, 5.2 and the OBBT experiments of Section 6)
and `oracle.scaling` (diagonal preconditioning in front of the same solver,
the problem scaling named in Section 2).

Pins: every function is checked in the CPU test suite against closed forms,
brute-force vertex enumeration, an independent LP solver (HiGHS via scipy),
Farkas' lemma for the infeasibility tests (rays of infeasible and unbounded
LPs are flagged; on feasible LPs the ratios stay above 1/||x^|| and 1/||c||),
first-order optimality of the proximal steps, firm nonexpansiveness, and
KKT/complementary-slackness invariants; the scaling against its own closed
forms (a diagonal matrix equilibrated in one pass, the Pock-Chambolle bound
||D_r A D_c|| <= 1) and objective invariance; the MIP outputs against exact
variable ranges and child optima from vertex enumeration and HiGHS; the
iterate trajectory without restarts against the worst-case rate bound of the
Halpern iteration; restarted trajectories (fixed weight, per LP and under the
batch-average scope) against what firm nonexpansiveness fixes across a
restart: each cycle starts no farther from a solution than the first, its
first residual is at most the one that fired the restart, and the rate bound
holds from its own start; the whole restarted trajectory against the scale
covariance of the LP (objective times alpha, box and rows times beta: the
iterates scale by beta and alpha exactly when the primal weight scales by
alpha / beta), which pins the form of the initial primal weight and the ratio
of the weight update.

Parity unpinned (readings no independent source fixes):
  * the exact restart times and iteration counts (the paper prints none);
  * the values of the restart constants beta_s, beta_n, beta_a, theta (named,
    not valued, in the paper);
  * the constant factor of the initial primal weight ||c|| / ||b|| and its
    fallback 1 below 1e-10 (the paper does not state w0; scale covariance
    fixes its form only up to a constant factor);
  * the strong-branching score weight mu = 1/6 of oracle.mip (the paper says
    only that the children's objectives determine the score; the value is
    the rule of the study it cites).
"""
from .lp import LP, row_bounds, from_arrays, from_instance, apply_delta, BASE, SET_LO, SET_HI, OBJ_UNIT
from .pdhg import (Options, Result, KKT, solve, solve_batch_avg, pdhg_operator,
                   fixed_point_residual, kkt, reduced_cost, proj_box, support,
                   proj_barrier_cone, proj_recession_cone, infeasibility, Infeasibility, opnorm, step_size, initial_primal_weight,
                   smoothed_primal_weight, restart_due,
                   RUNNING, OPTIMAL, ITERATION_LIMIT, INFEASIBLE_BOUNDS, NUMERICAL_ERROR,
                   PRIMAL_INFEASIBLE, DUAL_INFEASIBLE,
                   STATUS_NAMES)
