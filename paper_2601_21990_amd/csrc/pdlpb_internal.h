// Internal declarations shared by the gfx950 kernels (kernels.hip) and the
// C ABI implementation (pdlpb.cpp).  Not installed; the public interface is
// include/pdlpb.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdlpb {

// ---- per-slot state read by the fused step kernels ------------------------
// SLOT_FRESH marks an LP restarted by the last full evaluation: the plan of
// that evaluation copies z~ into its anchor and iterate, and the next residual
// evaluation records r(z^{n,0}) and clears the flag.  SLOT_RETIRE marks an LP
// that has stopped and whose results still sit in its slot; the next
// compaction copies them out and frees the slot.  SLOT_NEW marks an LP
// admitted into a running batch that has not made its first iteration yet.
enum : int32_t { SLOT_ACTIVE = 1, SLOT_FRESH = 2, SLOT_RETIRE = 4, SLOT_NEW = 8 };

// The per-slot state is stored as separate arrays so that the product kernels,
// which read it once per column per row, load 16 + 8 bytes per column: the key
// and the one step size they use.  The delta value is read only on the one row
// (variable) it changes.
struct SlotKey {
    int32_t t_anchor;  // global iteration index at which the current restart cycle began (k = t - t_anchor)
    int32_t t_end;     // global iteration index of the LP's last permitted iteration
    int32_t varkind;   // delta: variable | kind << 28 (PDLPB_BASE uses variable VAR_NONE)
    int32_t flags;     // SLOT_ACTIVE / SLOT_FRESH / SLOT_RETIRE
};
static_assert(sizeof(SlotKey) == 16, "SlotKey layout");
constexpr int32_t VAR_MASK = 0x0FFFFFFF;
constexpr int32_t VAR_NONE = 0x0FFFFFFF;   // no variable; n is limited to VAR_NONE - 1

struct Slots {          // all indexed by slot
    SlotKey* key;
    double*  tau;       // eta / w
    double*  sigma;     // eta * w
    double*  dval;      // delta value
    int32_t* t_start;   // global iteration index of the LP's first iteration
    int32_t* lp;        // LP held by the slot
};

// ---- per-LP control data (indexed by LP, not by slot) -----------------------
constexpr int RESTART_LOG = 64;
constexpr int MAX_BATCH = 4096;

struct SlotCtl {
    double  w;         // primal weight
    double  r0;        // residual at the start of the restart cycle
    double  r_prev;    // previous evaluated residual of the cycle; < 0 when none
    double  kkt[4];    // gap, primal, dual, max at the LP's last evaluation
    double  obj;       // c_j' x~
    double  dobj;      // dual objective -phi_box(r~) - phi_[l,u](y~) (eq:main_lp, dual side)
    int32_t status;    // PDLPB_STATUS_*
    int32_t iters;     // applications of T
    int32_t restarts;  // number of restarts
    int32_t t_last;    // global iteration index of the LP's last iteration
    int32_t k_last;    // inner index k of the LP's last iteration (Halpern weight of its last update)
    int32_t pad;
    double  tol;       // stopping tolerance of the LP (eq:stopping)
};

// ---- compaction plan written by the control pass, executed by k_compact ------
struct RetireEntry {
    int32_t slot;      // slot whose LP has stopped
    int32_t lp;        // that LP
    int32_t kp2;       // k_last + 2
    int32_t src;       // running slot beyond the new column count that moves into this
                       // slot once its results are copied out; -1 when none does
    double  a;         // (k_last + 1) / (k_last + 2)
    int32_t src_fresh; // 1: the moving LP restarted at this evaluation, so its anchor
                       // and dual iterate are its z~ (the move applies the restart)
    int32_t pad;
};
static_assert(sizeof(RetireEntry) == 32, "RetireEntry layout");
struct MoveEntry {
    int32_t src;       // running slot beyond the new column count
    int32_t dst;       // freed slot below it
};

// ---- batch-wide scalars on the device ---------------------------------------
struct Globals {
    int32_t t0;          // base iteration index of the current block of C iterations
    int32_t n_active;    // LPs still running after the last control pass
    int32_t batch_k0;    // BATCH_AVG: global index at which the shared restart cycle began
    int32_t n_cols;      // live columns: slots [0, n_cols) hold every running LP
    int32_t n_retire;    // compaction plan: stopped LPs to copy out
    int32_t n_move;      //   running LPs to move into freed slots
    int32_t n_cols_next; //   live columns after the compaction
    int32_t quiet;       // 1: the next evaluation that is not full has no LP to evaluate (no
                         //    running LP starts a restart cycle or reaches its last iteration)
    int32_t n_fresh;     // compaction plan: running LPs below n_cols_next that restarted at
                         //    this evaluation (their anchor and dual iterate become z~)
    int32_t pad;
    double  tol;
    double  eta;
    double  r0;          // BATCH_AVG shared r(z^{n,0})
    double  r_prev;      // BATCH_AVG shared previous residual (< 0: none)
};

// number of float64 sums each evaluation produces per LP and side
constexpr int NTERM = 10;
// x side: 0 |dx|^2, 1 c'x~, 2 phi_box(r~), 3 |c + A'y~ + r~|^2, 4 |c|^2, 5 |x~ - x0|^2,
//         6 phi_box(dr), 7 |A'dy_B + dr|^2, 8 c'dx, 9 |dx - Pi_R(dx)|^2
// y side: 0 |dy|^2, 1 dy'(A dx), 2 phi_[l,u](y~), 3 |Ax~ - Pi(Ax~)|^2, 4 |Ax~|^2, 5 |y~ - y0|^2,
//         6 phi_[l,u](dy_B), 7 |A dx - Pi_R(A dx)|^2, 8-9 unused
// (dy_B = Pi_B[l,u](dy), dr = Pi_B[xl,xu](r~ - r^k), the displacement vectors of the
// infeasibility tests)

template <typename T>
struct StepArgs {
    const int32_t* rp;   // CSR row pointers of the matrix whose rows this kernel walks
    const int32_t* ci;   // column indices
    const T*       av;   // values
    const int32_t* eci;  // ELL head: the first ew column indices of every row (-1 pads), rows x ew; may be null when ew = 0
    const T*       ev;   // ELL head values (0 pads)
    int32_t ew;          // ELL head width: 16, or 0 when the rows are walked in CSR alone
    int32_t rows;        // rows walked (n for the primal step, m for the dual step)
    int32_t ld;          // row stride of every dense block (>= ncols)
    int32_t ncols;       // columns covered by the grid (the live count g->n_cols never exceeds it)
    int32_t wpb;         // waves per block
    const T* G;          // block gathered by the product (Y for primal, Xbar for dual)
    T* Z;                // primal: Xbar (reflected x, 2x~ - x^k)   dual: Y (Halpern iterate y^k)
    T* Z0;               // anchor block X0 / Y0
    T* Zt;               // z~ block Xt / Yt (written on evaluation launches and final iterations)
    T* DZ;               // displacement z~ - z^k (same launches)
    const double* c;     // primal: base objective (n); dual: unused
    const double* lo;    // primal: base xl (n);  dual: row lower bounds l (m)
    const double* hi;    // primal: base xu (n);  dual: row upper bounds u (m)
    Slots sl;
    const Globals* g;
    int32_t it;          // iteration index inside the block; global t = g->t0 + it
    int32_t eval;        // 2: every running LP writes z~ and its displacement; 1: only the LPs
                         //    that the following evaluation of fresh cycles reads; 0: none
    int32_t admit;       // 1: only LPs flagged SLOT_NEW iterate (their first iteration)
    int32_t max_blocks;  // > 0: cap on the workgroups of the launch (waves then loop over rows)
};

template <typename T>
struct EvalArgs {
    int32_t n, m, ld, ncols;
    const int32_t* a_rp; const int32_t* a_ci; const T* a_v;    // A (m x n)
    const int32_t* t_rp; const int32_t* t_ci; const T* t_v;    // A' (n x m)
    const T *Xt, *DX, *X0, *Yt, *DY, *Y0;
    const double *c, *xl, *xu, *rl, *ru;
    const int8_t* rcode;     // per row of A: 1 if its lower bound is -inf, | 2 if its upper is +inf
    Slots sl;
    const Globals* g;        // live column count
    int32_t pw_x, pw_y;      // rows per wave on the x side / y side
    int32_t npx, npy;        // row panels (4 waves each) on each side
    double* part_x;          // [NTERM][ld][npx]
    double* part_y;          // [NTERM][ld][npy]
    int32_t it;              // iteration index inside the block; global t = g->t0 + it
    int32_t full;            // 1: every running LP's sums; 0: only LPs at the start of a
                             // restart cycle (k = 0) or at their last iteration need them
    int32_t kkt_only;        // 1 (with full = 1): a stopping test alone, whose control pass
                             // reads the terms of eq:stopping only (x side 1-4, y side 2-4):
                             // the displacement products are skipped and the other terms are 0
};

struct ControlArgs {
    int32_t ncols, ld, npx, npy;
    const double* part_x;
    const double* part_y;
    double* sums;            // [2*NTERM][ld] scratch written by the reduce kernel
    Slots sl;                // by slot
    SlotCtl* ctl;            // by LP
    int32_t* rlog;           // [LP][RESTART_LOG]
    RetireEntry* retire;     // compaction plan (>= B entries each)
    MoveEntry* moves;
    int32_t* fresh;          // slots of restarted LPs that stay in place
    Globals* g;
    int32_t it;              // iteration index inside the block
    int32_t full;            // 1: KKT and restart tests (t mod C == 0); 0: residual of fresh cycles only
    int32_t stop_only;       // 1 (with full = 0): the stopping test alone, at every LP (t mod S == 0)
    int32_t advance;         // 1: move g->t0 on by `block` after this pass
    int32_t block;           // C
    int32_t batch_avg;       // restart scope
    int32_t admit;           // 1: first evaluation of newly admitted LPs only
    int32_t admit_plan;      // with admit = 1: plan the compaction too, so admitted LPs that
                             //    stopped at once leave before the block's iterations
    int32_t pw_literal;      // primal weight ratio as printed
    double beta_s, beta_n, beta_a, theta, cross_sign;
    double infeas_tol;       // eps of the infeasibility tests; < 0: the stopping tolerance; 0: off
    double dual_tol;         // eps of the dual-feasibility test; < 0: the stopping tolerance
};

// Persistent tail: one workgroup per running LP iterates it to its stop.
constexpr int32_t TAIL_THREADS = 512;

template <typename T>
struct TailArgs {
    int32_t n, m, ld, C;
    int32_t S;                 // stopping tests also every S iterations of a block (0: off)
    int32_t ncols;             // workgroups: slots [0, ncols)
    const int32_t* a_rp; const int32_t* a_ci; const T* a_v;    // A (m x n)
    const int32_t* t_rp; const int32_t* t_ci; const T* t_v;    // A' (n x m)
    const int32_t* a_e8ci; const T* a_e8v;   // the first 8 entries of every row of A (-1 pads)
    const int32_t* t_e8ci; const T* t_e8v;   // ... and of A'
    T* blk[8];                 // Xbar, X0, Xt, DX, Y, Y0, Yt, DY (row-major, stride ld)
    T* res[4];                 // Rx, Rxi (B x n), Ry, Ryi (B x m): LP-major results
    const double *c, *xl, *xu, *rl, *ru;
    Slots sl;
    SlotCtl* ctl;
    int32_t* rlog;
    const Globals* g;          // t0 (base of the next block of C iterations) and eta
    ControlArgs ca;            // stopping, infeasibility and restart parameters
    int32_t pw_x, pw_y, npx, npy;
    T* work;                   // per workgroup: Xbar, X0, Xt, DX (n each), Y, Y0, Yt, DY (m each);
                               // Xbar and Y themselves live in LDS while the LP runs
    double* wsum;              // per workgroup: tail_sum_doubles(npx, npy) doubles
};
// LDS of the tail kernel: its evaluation terms (static) and Xbar, Y (dynamic)
constexpr size_t TAIL_STATIC_LDS = (size_t)TAIL_THREADS * (NTERM + 1) * sizeof(double) + 64;
__host__ __device__ inline size_t tail_sum_doubles(int32_t npx, int32_t npy) {
    // chain sums (4 per panel), panel values, the evaluation sums
    return (size_t)(4 * (npx + npy) + (npx + npy) + 2) * NTERM;
}

// ---- shared start ------------------------------------------------------------
// A batch whose running LPs all start from one warm point (or from zero), with
// the same step sizes for every LP of one base LP, makes its first iteration
// and evaluation (t = 0) once per base LP -- the LP without a change, and for
// objective changes that LP with objective 0 -- and per LP only where its
// change reaches: its variable v, the rows of A through v, and the evaluation
// rows that read them.
constexpr int32_t SP_MAX_COL = 64;       // nonzeros of a changed variable's column of A
constexpr int32_t SP_MAX_TOUCH = 4096;   // 1 + nonzeros of the rows of A through it
constexpr int32_t SP_SIDE = 4 + 3 * SP_MAX_COL;   // values of one LP where it differs

template <typename T>
struct SharedArgs {
    int32_t n, m, ld;
    int32_t nslots;            // running LPs: slots [0, nslots)
    int32_t ncls;              // base LPs (1 or 2)
    int32_t cls_kind[2];       // change kind of base LP K: PDLPB_BASE (objective c) or
                               // PDLPB_OBJ_UNIT (objective 0)
    int32_t cls_obj;           // base LP of the objective changes (-1: none in the batch)
    int32_t cls_bound;         // base LP of every other LP (-1: none)
    const int32_t* a_rp; const int32_t* a_ci; const T* a_v;    // A (m x n)
    const int32_t* t_rp; const int32_t* t_ci; const T* t_v;    // A' (n x m)
    const double *c, *xl, *xu, *rl, *ru;
    const int8_t* rcode;       // per row of A: 1 if its lower bound is -inf, | 2 if its upper is +inf
    const double *xw, *yw;     // the shared warm start (NULL: zero)
    double tau[2], sigma[2];   // step sizes of every LP of base LP K
    T *x0, *y0;                // x^0 on the base box (n), y^0 (m)
    T *xt, *xbar, *dx;         // [ncls][n]: x~, x-bar = 2 x~ - x^0, x~ - x^0 of each base LP
    T *yt, *yn, *dy;           // [ncls][m]: y~, y^1, y~ - y^0
    T* side;                   // [slot][SP_SIDE]: x^0, x~, x-bar, dx at v, then y~, y^1, dy
                               // at each row of A through v (in the order of A's column v)
    Slots sl;
    int32_t pw_x, pw_y, npx, npy;   // evaluation layout (as k_eval)
    double* rt;                // [ncls][n + m][NTERM]: terms of every row of each base LP
    double* bwave;             // [ncls][npx + npy][4][NTERM]: its chain sums
    double* bpanel;            // [ncls][npx + npy][NTERM]: its panel sums
    double* part_x;            // evaluation sums, laid out as k_eval writes them
    double* part_y;
    Globals* g;
    const RetireEntry* retire;
    const MoveEntry* moves;
    int32_t* map;              // [2][nslots]: slot whose LP a live column holds after the
                               // compaction, and that LP's base LP
    T* blk[8];                 // Xbar, X0, Xt, DX, Y, Y0, Yt, DY (row-major, stride ld)
    T* res[4];                 // Rx, Rxi (B x n), Ry, Ryi (B x m): LP-major results
};

// ---- launchers (kernels.hip) ---------------------------------------------------
// Each returns hipSuccess or the launch error.
template <typename T>
hipError_t launch_primal(const StepArgs<T>& a, int lanes, int vec, hipStream_t s);
template <typename T>
hipError_t launch_dual(const StepArgs<T>& a, int lanes, int vec, hipStream_t s);
template <typename T>
hipError_t launch_eval(const EvalArgs<T>& a, hipStream_t s);
hipError_t launch_reduce(const ControlArgs& a, hipStream_t s);
hipError_t launch_control(const ControlArgs& a, hipStream_t s);
// Iterate every running LP of slots [0, ncols) to its stop with one workgroup
// each, computing the same bits as the batched kernels (same products in CSR
// order, same evaluation chains and reduction trees, same control), and copy
// its results to the result blocks.
template <typename T>
hipError_t launch_tail(const TailArgs<T>& a, size_t dyn_lds, hipStream_t s);

// Shared start.  launch_sp_iterate: the first iteration (t = 0) of every base
// LP (x^0, x~, x-bar, dx; y^0, y~, y^1, dy), then of every LP at its variable
// and at the rows of A through it, as the step kernels compute them.
// launch_sp_eval: the evaluation sums at t = 0 of every running LP into
// part_x / part_y, the bits k_eval computes from the blocks.  launch_sp_place,
// after the control pass: the blocks Xbar, X0, Y, Y0 of the LPs that still
// run, at their slots after the compaction; the results of the stopped LPs;
// the slot state of moved LPs and the new column count (what k_compact does
// after a full evaluation; no LP restarts at t = 0).
template <typename T>
hipError_t launch_sp_iterate(const SharedArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_sp_eval(const SharedArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_sp_place(const SharedArgs<T>& a, hipStream_t s);

// Fill the iterate blocks of a new batch (Xbar = X0 = the projected warm x,
// Y = Y0 = the warm y).  Warm vectors: mode 0 none, 1 shared (xw: n, yw: m),
// 2 per LP (xw: ncols*n, yw: ncols*m, LP-major); slot_lp maps slots
// [0, ncols) to LPs (per-LP warm starts are indexed by LP).  The evaluation
// blocks (X~, dX, Y~, dY) are left as they are: a solve starts with a full
// evaluation, whose iteration writes them for every LP before anything reads
// them.
template <typename T>
hipError_t launch_init_blocks(int32_t n, int32_t m, int32_t ld, int32_t ncols, Slots sl,
                              const double* xl, const double* xu, const double* xw,
                              const double* yw, int32_t mode, T* Xbar, T* X0, T* Y, T* Y0,
                              hipStream_t s);

// Execute the plan of a full evaluation in one launch: restarted LPs take z~
// as anchor and dual iterate (Section 4, restarts), stopped LPs' z~ and last
// Halpern iterate are copied into the LP-major result blocks, and running LPs
// beyond the new column count move into the freed slots.  ncols bounds the
// plan's entries (the live column count of the launches).
// blk: Xbar, X0, Xt, DX, Y, Y0, Yt, DY (row-major, stride ld).
// res: Rx (B x n), Rxi (B x n), Ry (B x m), Ryi (B x m), LP-major.
template <typename T>
hipError_t launch_compact(int32_t n, int32_t m, int32_t ld, int32_t ncols, T* const* blk,
                          T* const* res, const RetireEntry* retire, const MoveEntry* moves,
                          const int32_t* fresh, Slots sl, Globals* g, hipStream_t s);

// Start a solve: t_end of every live slot from the iteration budget, g->t0 = 0.
hipError_t launch_begin_solve(Slots sl, SlotCtl* ctl, int32_t ncols, int32_t max_iters, Globals* g,
                              double tol, hipStream_t s);

// Initialise columns [c0, c0 + cnt) of the eight blocks for newly admitted LPs
// (warm start: PDLPB_WARM_NONE, or PDLPB_WARM_BASE from the base vectors
// xw (n) / yw (m), where objective changes take xw and y = 0).
template <typename T>
hipError_t launch_init_columns(int32_t n, int32_t m, int32_t ld, int32_t c0, int32_t cnt, Slots sl,
                               const double* xl, const double* xu, const double* xw,
                               const double* yw, int32_t mode, T* const* blk, hipStream_t s);

// ctl[rows[i]] = src[i] for i < cnt; g->n_cols = n_cols.
hipError_t launch_admit(SlotCtl* ctl, const int32_t* rows, const SlotCtl* src, int32_t cnt,
                        Globals* g, int32_t n_cols, hipStream_t s);

// Convert n entries of a result block to float64 (FP32 mode).
hipError_t launch_widen(const float* src, int64_t count, double* dst, hipStream_t s);

// v[k] *= d[k % period], or v[k] /= d[k % period] when divide != 0.
hipError_t launch_rescale(double* v, const double* d, int64_t count, int32_t period,
                          int32_t divide, hipStream_t s);

// Power iteration building blocks (float64, one vector).
hipError_t launch_spmv(const int32_t* rp, const int32_t* ci, const double* v, int32_t rows,
                       const double* x, double* y, hipStream_t s);
// sum of squares of x (length len) -> *out, deterministic two-pass; partial holds >= 1024 doubles
hipError_t launch_norm2sq(const double* x, int32_t len, double* partial, double* out,
                          hipStream_t s);
hipError_t launch_scale(double* x, int32_t len, const double* nrm2sq, hipStream_t s);
hipError_t launch_fill(double* x, int32_t len, double v, hipStream_t s);

}  // namespace pdlpb
