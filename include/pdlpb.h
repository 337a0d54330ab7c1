/*
 * pdlpb.h -- batched restarted PDHG for many LPs that share one constraint
 * matrix, on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Method: arXiv 2601.21990, "Batched First-Order Methods for Parallel LP
 * Solving in MIP".  Every LP of a batch is
 *
 *     min c_j'x   s.t.   l <= A x <= u,   xl_j <= x <= xu_j        (eq:main_lp, Section 3)
 *
 * with A, l, u shared by the whole batch and c_j, xl_j, xu_j equal to the base
 * vectors except for one change per LP: a raised lower bound or lowered upper
 * bound of one variable (full strong branching, Section 5.1) or the objective
 * +-e_var (bound tightening, Section 5.2).  The batch is solved together by the
 * reflected Halpern PDHG iteration with adaptive restarts (Section 4; batched
 * form eq:batched_iter and eq:main-iterate, Section 5): each iteration is one
 * sparse-matrix times dense-block product with A' and one with A, fused with
 * the per-LP projection, reflection and averaging steps.
 *
 * Conventions
 *   - Row bounds come from a right-hand side b and one sense byte per row:
 *     'E' (l = u = b), 'L' (A x <= b), 'G' (A x >= b), 'N' (free row).
 *   - Dual signs follow the paper's saddle function c'x + y'Ax - phi_[l,u](y)
 *     (eq:lp_saddle): y_i >= 0 on an 'L' row, y_i <= 0 on a 'G' row.
 *   - Dense vectors of one LP are contiguous float64 arrays (x: n, y: m).
 *     Per-LP blocks passed or returned for a whole batch are LP-major: LP j
 *     occupies elements [j*n, (j+1)*n) (resp. [j*m, (j+1)*m)).
 *   - All pointer arguments are host memory unless a `mem` argument says
 *     PDLPB_MEM_DEVICE, in which case they are device pointers on the
 *     context's GPU.  Inputs are copied during the call; the caller keeps
 *     ownership and may free them on return.  The context owns every device
 *     buffer it allocates.
 *   - Every call returns PDLPB_OK (0) or a negative error code and never
 *     throws.  pdlpb_last_error() describes the last failure.  Solver outcomes
 *     of single LPs are statuses (PDLPB_STATUS_*), not errors.
 *   - A context is not thread-safe; distinct contexts may be used from
 *     distinct threads.
 */
#ifndef PDLPB_H
#define PDLPB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define PDLPB_OK        0
#define PDLPB_EINVAL   (-1)   /* malformed argument: bad CSR, NaN data, unknown sense, B <= 0, var out of range */
#define PDLPB_ENOMEM   (-2)   /* device or host allocation failed, or the batch exceeds the capacity limit */
#define PDLPB_EDEVICE  (-3)   /* a HIP runtime call failed (no GPU, launch failure, ...) */
#define PDLPB_ESTATE   (-4)   /* call out of order, e.g. solve before set_batch */

/* ---- per-LP statuses -------------------------------------------------- */
#define PDLPB_STATUS_RUNNING            0
#define PDLPB_STATUS_OPTIMAL            1  /* max(gap, primal, dual) <= tol (eq:stopping) at an evaluation */
#define PDLPB_STATUS_ITERATION_LIMIT    2  /* max_iters applications of T without meeting tol */
#define PDLPB_STATUS_INFEASIBLE_BOUNDS  3  /* the LP's change crosses its variable bounds (xl > xu); never iterated */
#define PDLPB_STATUS_NUMERICAL_ERROR    4  /* a NaN or infinity reached the residual or the KKT measures */
#define PDLPB_STATUS_INVALID_INPUT      5  /* the LP's change carries NaN, or +inf as a lower / -inf as an upper bound */
#define PDLPB_STATUS_PRIMAL_INFEASIBLE  6  /* the primal infeasibility test passed (eq:primal-infeas, Section 4) */
#define PDLPB_STATUS_DUAL_INFEASIBLE    7  /* the dual infeasibility test passed (eq:dual-infeas): the LP is unbounded or infeasible */

/* ---- per-LP change ("delta") ------------------------------------------- */
#define PDLPB_BASE      0   /* the base LP itself */
#define PDLPB_SET_LO    1   /* xl[var] = value  (branch up: value = ceil(x_rel[var]), Section 5.1) */
#define PDLPB_SET_HI    2   /* xu[var] = value  (branch down: value = floor(x_rel[var]), Section 5.1) */
#define PDLPB_OBJ_UNIT  3   /* c = value * e_var (bound tightening: +1 minimises, -1 maximises x_var, Section 5.2) */

typedef struct pdlpb_delta {
    int32_t kind;      /* PDLPB_BASE / PDLPB_SET_LO / PDLPB_SET_HI / PDLPB_OBJ_UNIT */
    int32_t var;       /* variable index in [0, n); ignored for PDLPB_BASE */
    double  value;
} pdlpb_delta;         /* 16 bytes, no padding */

/* ---- options ----------------------------------------------------------- */
#define PDLPB_FP64      0   /* A, iterates and products in float64 */
#define PDLPB_MIXED32   1   /* A (rounded), iterates and products in float32; residual, KKT and restart sums in float64 */

#define PDLPB_RESTART_PER_LP     0  /* each LP applies the restart tests to its own residual */
#define PDLPB_RESTART_BATCH_AVG  1  /* restart tests on the batch-average residual, all LPs restart together (Section 5) */

#define PDLPB_WARM_NONE    0   /* x = projection of 0 onto the LP's box, y = 0 */
#define PDLPB_WARM_SHARED  1   /* one x (n) and y (m) for every LP, projected onto each LP's box */
#define PDLPB_WARM_PER_LP  2   /* LP-major blocks x (B*n) and y (B*m) */
#define PDLPB_WARM_BASE    3   /* serving: the context's resident warm start (pdlpb_set_base_warm) */

#define PDLPB_MEM_HOST     0
#define PDLPB_MEM_DEVICE   1

typedef struct pdlpb_options {
    int32_t struct_size;      /* sizeof(pdlpb_options); set by pdlpb_default_options */
    int32_t precision;        /* PDLPB_FP64 (default) or PDLPB_MIXED32 */
    int32_t restart_scope;    /* PDLPB_RESTART_PER_LP (default) or PDLPB_RESTART_BATCH_AVG */
    int32_t eval_every;       /* C: residual, KKT and restart tests every C iterations (default 64) */
    double  beta_sufficient;  /* restart when r <= beta_s r0                      (default 0.2)  */
    double  beta_necessary;   /* ... or r <= beta_n r0 and r grew since last test (default 0.8)  */
    double  beta_artificial;  /* ... or k > beta_a * iterations so far            (default 0.36) */
    double  theta;            /* primal-weight smoothing exponent                 (default 0.5)  */
    double  step_size;        /* eta; 0 (default) computes 0.998 / ||A||_2 (Section 4) */
    double  cross_sign;       /* sign s of the off-diagonal blocks of the residual metric M (default -1) */
    double  infeas_tol;       /* eps of the infeasibility tests at each evaluation: < 0 (default -1) uses the
                                 stopping tolerance of pdlpb_solve, 0 disables them, > 0 as given */
    int32_t pw_ratio;         /* 0 (default): d = ||dy||/||dx||; 1: d = ||dx||/||dy|| as printed */
    int32_t device;           /* HIP device ordinal (default 0) */
    void*   stream;           /* hipStream_t to run on; NULL = a stream owned by the context */
    int32_t max_batch;        /* largest B accepted by set_batch (default 4096) */
    int32_t use_graphs;       /* 1 (default): replay each block of C iterations as one captured hipGraph */
    int32_t tile_lanes;       /* 0 = automatic; else lanes per row group of the fused SpMM kernels (1..64, power of 2) */
    int32_t tile_vec;         /* 0 = automatic; else columns per lane (1, 2 or 4) */
    int32_t autotune;         /* 1 (default): time tile shapes on the first block of C iterations of
                                 a large batch and keep the fastest per kernel; 0: fixed heuristic */
    int32_t shared_start;     /* first iteration of a batch whose running LPs all start from one point
                                 (PDLPB_WARM_NONE or PDLPB_WARM_SHARED), the objective changes with
                                 one primal weight and the other LPs with one primal weight
                                 (Section 5: the LPs differ from a common LP in one variable): it is
                                 made once for the common LP (and once for it with objective 0 when
                                 the batch holds objective changes) and per LP only at its variable
                                 and the rows of A through it; the evaluation at t = 0 likewise; the
                                 dense blocks are then written only for the LPs still running.  The
                                 results are those of the full-width path, bit for bit.  0 (default):
                                 when the batch's blocks hold at least 256 MB (one block pair over
                                 the running LPs); 1: whenever the batch
                                 qualifies; -1: never.  A change qualifies when its variable's
                                 column has at most 64 nonzeros and the rows through it at most
                                 4095 in all */
    double  dual_tol;         /* eps of the dual-feasibility test of eq:stopping: < 0 (default -1) uses the
                                 stopping tolerance; >= 0 as given.  The bound-tightening experiments of
                                 Section 6 check dual feasibility at 1e-8 before trusting a dual bound */
    int32_t max_blocks;       /* cap on the workgroups of one step launch; their waves loop over the rows.
                                 0 (default): 16384 (64 4-wave workgroups per compute unit) */
    int32_t scaling;          /* diagonal preconditioning of A at create: 0 (default) none; 1 ten Ruiz
                                 equilibration passes then one Pock-Chambolle pass (alpha = 1).  The
                                 solver then works on D_r A D_c (the stopping and infeasibility tests
                                 measure the scaled LP); changes, warm starts and results stay in the
                                 caller's coordinates */
    int32_t tail_cols;        /* persistent tail: once at most this many LPs of a batch still run
                                 (0, the default, disables), on a matrix of at most 65536 nonzeros and
                                 with the per-LP restart scope, pdlpb_solve finishes them in one
                                 launch with one workgroup per LP, which computes the same bits as
                                 the batched kernels (Section 5: the LPs left once most have stopped).
                                 One CU then streams the whole matrix every iteration: it is faster
                                 than the batched kernels only on matrices of a few thousand
                                 nonzeros, so it is left to the caller */
    int32_t stop_every;       /* S: the stopping test (eq:stopping at z~) also runs every S
                                 iterations between the evaluations of eval_every (Section 4 leaves
                                 the schedule open); it tests nothing else, so the iterates are
                                 those of the run without it and LPs only stop sooner.  0 (the
                                 default) or eval_every: off; otherwise a divisor >= 2 of
                                 eval_every.  Per-LP restart scope, pdlpb_solve only (ignored by
                                 the serving calls). */
    /* Device memory of the context.  Both NULL (default): hipMalloc / hipFree.
       Otherwise both set: every device buffer the context holds comes from
       dev_alloc(bytes, alloc_user), which returns a pointer on the context's
       device aligned to at least 256 bytes, or NULL (the call that needed it
       then fails with PDLPB_ENOMEM), and goes back through
       dev_free(ptr, bytes, alloc_user) with the size it was requested with.
       The context synchronises its stream before each dev_free, so memory
       handed back is no longer in use.  A caching allocator (such as
       PyTorch's) can back a context this way.  Buffers are requested by
       pdlpb_create, by calls whose batch outgrows the storage (set_batch,
       serve_begin, estimate_batch) and by result copies that need staging;
       they are returned when storage is replaced and by pdlpb_destroy. */
    void* (*dev_alloc)(size_t bytes, void* alloc_user);
    void  (*dev_free)(void* ptr, size_t bytes, void* alloc_user);
    void*  alloc_user;
} pdlpb_options;

typedef struct pdlpb_ctx pdlpb_ctx;   /* opaque; owns all device memory of one base matrix and its batch */

/* Fill *opt with the defaults listed above. */
void pdlpb_default_options(pdlpb_options* opt);

/*
 * Create a context for one constraint matrix and base LP (eq:main_lp).
 *   A: m x n in CSR -- row_ptr (m+1 entries, row_ptr[0] = 0, nondecreasing,
 *      row_ptr[m] = nnz), col_idx (nnz, strictly increasing inside each row,
 *      in [0, n)), val (nnz, finite).  m >= 0, n >= 1, nnz < 2^31.
 *   c (n, finite), b (m, finite; unused by 'N' rows), sense (m bytes from
 *   "ELGN"), l / u (n variable bounds; -inf / +inf allowed, l <= u, NaN not).
 *   opt: NULL for defaults.
 * Copies A and A' to the GPU once and computes the step size
 * eta = 0.998 / ||A||_2 by power iteration (Section 4) unless opt->step_size > 0.
 * Returns PDLPB_EINVAL (nothing allocated, *out = NULL) on malformed input.
 */
int pdlpb_create(pdlpb_ctx** out, int32_t m, int32_t n, int64_t nnz,
                 const int64_t* row_ptr, const int32_t* col_idx, const double* val,
                 const double* c, const double* b, const char* sense,
                 const double* l, const double* u, const pdlpb_options* opt);

/*
 * Define a batch of B LPs, one change each (Section 5; strong branching 5.1,
 * bound tightening 5.2).  deltas: B entries.  Warm start per warm_mode:
 *   NONE: x_warm, y_warm ignored;  SHARED: x_warm (n), y_warm (m);
 *   PER_LP: x_warm (B*n), y_warm (B*m), LP-major.
 * w_warm: NULL (initial primal weight ||c_j|| / ||b||, or 1 when either is
 * below 1e-10), else B initial primal weights (> 0, finite).
 * mem: PDLPB_MEM_HOST or PDLPB_MEM_DEVICE for deltas, x_warm, y_warm, w_warm.
 * An LP whose change crosses its bounds gets PDLPB_STATUS_INFEASIBLE_BOUNDS,
 * one whose change is not a number gets PDLPB_STATUS_INVALID_INPUT; neither
 * is iterated and neither affects the others.  A kind outside 0..3 or a var
 * outside [0, n) fails the call with PDLPB_EINVAL.  Device storage grows to
 * the largest B seen and is reused for smaller batches.  A batch ends any
 * serving session on the context (its queued requests and results are
 * dropped; pdlpb_serve_begin starts a new one).
 */
int pdlpb_set_batch(pdlpb_ctx* ctx, int32_t B, const pdlpb_delta* deltas,
                    const double* x_warm, const double* y_warm, const double* w_warm,
                    int32_t warm_mode, int32_t mem);

/*
 * Iterate every LP of the current batch until it is OPTIMAL (relative KKT
 * measure <= tol at an evaluation, eq:stopping), or is detected
 * PRIMAL_INFEASIBLE / DUAL_INFEASIBLE (Section 4, tested at each evaluation
 * after the stopping test), or has applied the PDHG operator max_iters times
 * (ITERATION_LIMIT), or fails (NUMERICAL_ERROR).
 * tol >= 0, max_iters >= 1.  All control (restarts, primal weights, statuses)
 * runs on the GPU; the host only checks once per C iterations whether any LP
 * is still running (in a long solve of small launches the device runs one
 * block of C iterations ahead of that check; a block that finds every LP
 * stopped does nothing).  The call returns once every LP has stopped, with no
 * work of its own left on the context's stream.  Returns PDLPB_ESTATE if no
 * batch is set or it was already solved.
 */
int pdlpb_solve(pdlpb_ctx* ctx, double tol, int64_t max_iters);

/*
 * Results of LP j (0 <= j < B, in set_batch order) after pdlpb_solve.
 * x (n) and y (m) receive z~ = T(z) of the LP's last iteration, the point at
 * which the KKT measures are taken; either may be NULL.  kkt receives
 * {gap, primal, dual, max} (eq:stopping), obj receives c_j'x.  Any output
 * pointer may be NULL.  mem selects where x and y live.
 */
int pdlpb_get(pdlpb_ctx* ctx, int32_t j, double* x, double* y, int32_t* status,
              double kkt[4], double* obj, int64_t* iters, int32_t mem);

/*
 * Result blocks of the caller for the batches that follow: X (capacity x n
 * doubles) and Y (capacity x m doubles), LP-major device memory on the
 * context's device.  pdlpb_solve then writes every LP's x~ and y~ there as it
 * stops (LPs that never run get zeros at pdlpb_set_batch), instead of into
 * the context's own result blocks, so that pdlpb_get_batch into the same
 * pointers copies nothing (pdlpb_get, pdlpb_get_batch into other memory and
 * pdlpb_get_batch_noalloc read them from there).  The caller must keep them
 * valid and must not write them while a batch is set.  FP64 contexts without
 * scaling only.  Both NULL returns to the context's own blocks.  Either way
 * the current batch is dropped (call pdlpb_set_batch again).  Serving ignores
 * them.  EINVAL: one pointer NULL, an FP32 or scaled context, capacity
 * outside [1, max_batch]; pdlpb_set_batch then refuses a batch of more than
 * capacity LPs (EINVAL).
 */
int pdlpb_set_result_buffers(pdlpb_ctx* ctx, double* X, double* Y, int32_t capacity);

/*
 * Results of the whole batch at once: X (B*n) and Y (B*m) LP-major, status
 * (B), kkt (4*B: gap, primal, dual, max per LP), obj (B), iters (B).  Any
 * pointer may be NULL.  mem applies to X and Y; the per-LP arrays are host.
 */
int pdlpb_get_batch(pdlpb_ctx* ctx, double* X, double* Y, int32_t* status, double* kkt,
                    double* obj, int64_t* iters, int32_t mem);

/*
 * Diagnostics of LP j: the reflected Halpern iterate z^{k+1} produced by the
 * LP's last iteration (eq:mainiter) in x_iter (n) / y_iter (m), its final
 * primal weight w, its number of restarts, and up to log_cap iteration
 * indices at which it restarted (restart_log).  Any pointer may be NULL.
 */
int pdlpb_get_trace(pdlpb_ctx* ctx, int32_t j, double* x_iter, double* y_iter, double* w,
                    int32_t* restarts, int32_t* restart_log, int32_t log_cap);

/*
 * pdlpb_get_batch for callers that cannot allocate device memory (code that
 * must not call hipMalloc, such as tight serving loops or work recorded into
 * a HIP graph).  Same arguments, results and errors as pdlpb_get_batch, and
 * it allocates nothing: pdlpb_get_batch stages host copies that need FP32
 * widening (PDLPB_MIXED32) or the scaling (pdlpb_options.scaling) in a device
 * buffer it allocates, while this call stages them in a fixed array of
 * PDLPB_NOALLOC_SCRATCH_BYTES per GPU, set up by pdlpb_create and held until
 * the process ends, as many LPs at a time as fit.  Device destinations and
 * FP64 unscaled contexts need no staging.  Fails with PDLPB_EINVAL when
 * staging is needed and one LP's vector (n or m doubles) does not fit the
 * array.  The array is shared by every context on a GPU and keeps the last
 * call's contents; overlapping calls would race on it, so the library runs
 * calls of this entry point one at a time within a process (each process has
 * its own array).
 */
#define PDLPB_NOALLOC_SCRATCH_BYTES (32u << 20)
int pdlpb_get_batch_noalloc(pdlpb_ctx* ctx, double* X, double* Y, int32_t* status, double* kkt,
                            double* obj, int64_t* iters, int32_t mem);

/*
 * Dual objective -phi_box(r~) - phi_[l,u](y~) of every LP of the solved batch
 * (the dual of eq:main_lp, with r~ the reduced cost of Section 4) at the point
 * its KKT measures were taken: dual_obj (B host doubles).  For an LP whose
 * box is finite it is a lower bound on the LP's optimum by weak duality.
 * NaN for LPs that never iterated.  ESTATE before pdlpb_solve.
 */
int pdlpb_get_dual_objective(pdlpb_ctx* ctx, double* dual_obj);

/*
 * Bound tightening (Section 5.2) with the safeguards of the OBBT experiments
 * (Section 6): every OBJ_UNIT LP j of the solved batch minimised v_j x_var
 * (v_j = its value).  If it stopped OPTIMAL, its safe bound is
 * (D_j - Delta_j) / v_j, with D_j its dual objective and
 * Delta_j = eps (1 + |c_j'x~| + |D_j|): a lower bound on x_var if v_j > 0, an
 * upper bound if v_j < 0.  lo / hi (n host doubles, written) start as the base
 * bounds; a bound is replaced only if the new value improves it by more than
 * min_improve (the experiments use eps = 1e-8 with pdlpb_options.dual_tol =
 * 1e-8, and min_improve = 1e-4).  LPs are applied in batch order, each
 * compared with the running value.  *n_changed (may be NULL) counts replacements;
 * *infeasible (may be NULL) is 1 if some OBJ_UNIT LP stopped
 * PDLPB_STATUS_PRIMAL_INFEASIBLE, i.e. the shared feasible set is empty.
 * LPs that hit the iteration limit or failed give no bound.  Other change
 * kinds are ignored.  EINVAL: NULL lo/hi, eps or min_improve negative or not
 * finite.  ESTATE before pdlpb_solve.
 */
int pdlpb_obbt_tighten(pdlpb_ctx* ctx, double eps, double min_improve, double* lo, double* hi,
                       int32_t* n_changed, int32_t* infeasible);

/*
 * Strong-branching scores (Section 5.1) of the solved batch.  gain (B host
 * doubles, may be NULL): for a SET_LO (up) or SET_HI (down) LP that stopped
 * OPTIMAL, max(c'x~ - parent_obj, 0); +inf if it stopped primal infeasible or
 * its change crossed the variable's bounds; NaN otherwise and for other change
 * kinds.  score (B host doubles, may be NULL): for each such LP, the score of
 * its variable, (1 - mu) min(g_down, g_up) + mu max(g_down, g_up) (+inf if
 * either gain is), with g_down / g_up the gains of the first SET_HI / SET_LO
 * LP on that variable in batch order; NaN if either gain is NaN or the
 * variable has no opposite branch in the batch.  mu = 1/6 is the weight of the
 * scoring rule the paper cites.  EINVAL: parent_obj not finite, mu outside
 * [0, 1].  ESTATE before pdlpb_solve.
 */
int pdlpb_branch_scores(pdlpb_ctx* ctx, double parent_obj, double mu, double* gain, double* score);

/*
 * Serving: continuous batching of LPs on one resident matrix.
 *
 * pdlpb_serve_begin switches a context to serving with at most max_batch LP
 * columns and at most `result_capacity` result rows.  pdlpb_submit queues LPs
 * (one change each, as in pdlpb_set_batch) with their own tolerance and
 * iteration budget and returns consecutive ids; it fails with PDLPB_ENOMEM
 * when fewer than `count` result rows are free (pdlpb_release frees them).
 * Each pdlpb_serve_launch admits queued LPs into free columns (FIFO; the
 * admitted LPs make their first iteration, an evaluation, at admission) and
 * enqueues one block of C iterations for every running LP without waiting for
 * it; pdlpb_serve_wait waits for that block and records which LPs stopped.
 * With the per-LP restart scope every LP follows the same iteration schedule
 * from its own first iteration, so its result does not depend on when it was
 * admitted or on the LPs beside it.  Launch/wait pairs of several contexts
 * overlap on the device (each context has its own stream).
 *
 * Device storage follows the admitted work: a session starts with one column
 * and one result row, and pdlpb_serve_launch grows both (to the next power of
 * two, within the limits above) so that every running and queued LP has a
 * column and every row in use exists, moving the running LPs' columns into
 * the new storage.  pdlpb_serve_footprint tells a caller the device bytes the
 * context will hold once `extra` more LPs are submitted, so that a loop over
 * several contexts can admit a request only when its footprint fits one
 * device-memory budget; pdlpb_serve_trim shrinks the storage to what the LPs
 * still queued, running or holding result rows need.
 *
 * pdlpb_set_base_warm keeps one warm start (x: n, y: m, primal weight w)
 * resident on the device for PDLPB_WARM_BASE submissions.  A bound change
 * (SET_LO / SET_HI) starts from the base x (projected onto its box), y and w.
 * An objective change (OBJ_UNIT) starts from the base x with y = 0 and the
 * default weight ||c_j|| / ||b||: the base dual and weight belong to the base
 * objective, and starting from them stalls FP32 iterates far from the optimum.
 */
int pdlpb_set_base_warm(pdlpb_ctx* ctx, const double* x, const double* y, double w, int32_t mem);
int pdlpb_serve_begin(pdlpb_ctx* ctx, int32_t result_capacity);
int pdlpb_submit(pdlpb_ctx* ctx, int32_t count, const pdlpb_delta* deltas, int32_t warm_mode,
                 double tol, int64_t max_iters, int32_t mem, int64_t* first_id);
int pdlpb_serve_launch(pdlpb_ctx* ctx);
int pdlpb_serve_wait(pdlpb_ctx* ctx, int32_t* n_running, int32_t* n_queued);
/* Ids of LPs that stopped since the last poll (at most cap); *count receives how many. */
int pdlpb_poll(pdlpb_ctx* ctx, int64_t* ids, int32_t cap, int32_t* count);
/*
 * Result of a submitted LP (as pdlpb_get).  Until the LP has stopped (its id
 * was returned by pdlpb_poll, or it settled at submission) the call reports
 * status PDLPB_STATUS_RUNNING, kkt and obj NaN and iters 0, and writes
 * neither x nor y.  EINVAL for an unknown or released id.
 */
int pdlpb_result(pdlpb_ctx* ctx, int64_t id, double* x, double* y, int32_t* status,
                 double kkt[4], double* obj, int64_t* iters, int32_t mem);
/* Free the result row of a stopped LP; its id becomes invalid.  PDLPB_ESTATE
 * while the LP is queued or running (its row is still in use). */
int pdlpb_release(pdlpb_ctx* ctx, int64_t id);
/*
 * 1 when no block of the session is in flight or the last one launched has
 * finished on the device (pdlpb_serve_wait will not block), 0 while it still
 * runs, a negative error code on a device error.  Never blocks, so a loop can
 * serve the contexts whose blocks finish first.
 */
int pdlpb_serve_ready(pdlpb_ctx* ctx);
/*
 * *bytes = device bytes the context will hold (pdlpb_device_bytes: matrix,
 * base vectors, warm start and batch storage) once `extra` (>= 0) more LPs
 * are submitted and admitted, with the storage grown as pdlpb_serve_launch
 * grows it.  With extra = 0: what its running and queued LPs will hold.
 */
int pdlpb_serve_footprint(pdlpb_ctx* ctx, int32_t extra, int64_t* bytes);
/*
 * Shrink the session's storage to the next power of two at or above what its
 * running and queued LPs (columns) and its rows in use need, keeping their
 * data.  PDLPB_ESTATE while a block is in flight.
 */
int pdlpb_serve_trim(pdlpb_ctx* ctx);

/*
 * Batch width estimate (Section 5, "Matrix-matrix products and optimal batch
 * size"): the paper times ten products A X and ten products A'Y at several
 * batch widths before a MIP solve and takes the width that maximises the
 * matrix-vector products per second.  For each widths[i] this runs `reps`
 * fused primal steps (A'Y) and `reps` fused dual steps (A Xbar) of the
 * context's own kernels on a batch of widths[i] copies of the base LP (after
 * one untimed pair), timed with HIP events on the context's stream.  ms
 * (count host doubles, may be NULL) receives the elapsed milliseconds per
 * width; *best (may be NULL) the width with the most column products per
 * second, 2 reps widths[i] / ms[i] (the first of equal ones).  The call
 * replaces the context's batch: a batch set before it, its results and any
 * serving session end.  Storage grows to the largest width.  EINVAL: NULL
 * widths, count < 1, reps outside [1, 1000], a width outside [1, max_batch].
 */
int pdlpb_estimate_batch(pdlpb_ctx* ctx, const int32_t* widths, int32_t count, int32_t reps,
                         double* ms, int32_t* best);

/*
 * Tile shape of the fused product kernels for the following pdlpb_set_batch
 * calls: `lanes` lanes (1..64, power of two) per row group, `vec` consecutive
 * LPs (1, 2 or 4) per lane, so one group covers lanes*vec LPs of a row and a
 * wave covers 64/lanes rows.  lanes = vec = 0 restores the automatic choice.
 * Every shape sums each row in the same order, so results do not change.
 */
int pdlpb_set_tile(pdlpb_ctx* ctx, int32_t lanes, int32_t vec);

/*
 * The diagonal scaling in use (pdlpb_options.scaling): dr (m host doubles) and
 * dc (n host doubles) with the solver's matrix D_r A D_c; all ones without
 * scaling.  Either pointer may be NULL.  Problem scaling is one of the
 * enhancements of the first-order method the paper builds on (Section 2).
 */
int pdlpb_get_scaling(const pdlpb_ctx* ctx, double* dr, double* dc);

/* Step size eta in use and the computed ||A||_2 (0 if eta was given). */
int pdlpb_get_step_size(const pdlpb_ctx* ctx, double* eta, double* norm_a);

/*
 * Kernel timing.  While enabled, pdlpb_solve runs without graph replay and
 * brackets every launch of the fused SpMM kernels with HIP events on the
 * context's stream.  pdlpb_kernel_times reports, per kind
 * (0: A'Y + primal step, 1: A X + dual step, 2: evaluation, 3: control,
 * restarts and compaction, 4: persistent tail), the number of launches and
 * their summed duration in milliseconds since the last reset.
 */
int pdlpb_set_kernel_timing(pdlpb_ctx* ctx, int32_t enable);
int pdlpb_kernel_times(pdlpb_ctx* ctx, int64_t counts[5], double total_ms[5]);

/*
 * For the same launches: the live LP columns each launch processed, summed
 * per kind (the live count is read back at every evaluation; within a block
 * of C iterations it does not change).  Algorithmic bytes of the product
 * kernels are affine in the column count, so with the launch count this gives
 * their exact sum.  EINVAL for a NULL cols.
 */
int pdlpb_kernel_columns(pdlpb_ctx* ctx, int64_t cols[5]);

/* Bytes of device memory held by the context.  Besides the matrix, base
 * vectors, batch storage and results, a context that has solved a batch whose
 * eight blocks exceed the last-level cache (n + m rows at its stride, at least
 * 256 MB per pair of blocks) keeps eight blocks each of 16, 4, 2 and 1
 * columns, (n + m) * 23 * element size * 4 bytes in all, where a batch's last
 * LPs finish (Section 5: the LPs left once most have stopped); one whose batch
 * took the shared start (option shared_start) keeps its base vectors,
 * (n + m)(1 + 3K) elements for K <= 2 base LPs, 196 elements per LP column,
 * and 80 (n + m) K bytes of evaluation terms; pdlpb_serve_begin releases
 * both. */
int64_t pdlpb_device_bytes(const pdlpb_ctx* ctx);

/* Number of blocks of C iterations captured as graphs over the context's life.
 * A captured block is replayed for every later batch or serving round with the
 * same launch shape (live column bound, row stride, tile shapes, the batch's
 * blocks or those of 16, 4, 2 or 1 columns, the result blocks written), and is
 * captured again only when the context's storage is reallocated. */
int64_t pdlpb_graph_captures(const pdlpb_ctx* ctx);

/* Release every device buffer and the context.  NULL is a no-op. */
void pdlpb_destroy(pdlpb_ctx* ctx);

/*
 * Message for the last failed call on ctx, or for the last failed
 * pdlpb_create on this thread when ctx is NULL.  Never NULL; valid until the
 * next call on the same context (or thread).
 */
const char* pdlpb_last_error(const pdlpb_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* PDLPB_H */
