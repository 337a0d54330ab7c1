// C ABI of the batched restarted PDHG solver: argument validation, device
// memory, the step size, batch set-up, the host loop that replays blocks of C
// iterations, and result retrieval.  All arithmetic of an iteration runs in
// the kernels of kernels.hip; the host only checks, once per block, whether any
// LP is still running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "pdlpb.h"
#include "pdlpb_internal.h"

using namespace pdlpb;

namespace {

thread_local std::string g_create_error = "no error";

// ---- staging of pdlpb_get_batch_noalloc --------------------------------------
// A fixed device array instead of an allocation: each GPU the library runs on
// holds its own copy until the process ends.  Its name is not an address in
// host code; the address on each device comes from hipGetSymbolAddress, taken
// once per device (with that device current) when the first context is
// created there, and only that address is used on the host.
constexpr size_t NOALLOC_DOUBLES = (size_t)PDLPB_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;                   // guards the table and serialises the entry point
double* g_scratch_ptr[MAX_DEVICES] = {};   // address of the array on each device, once known

// Record the array's address on `device` (current).  Called by pdlpb_create.
hipError_t scratch_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
    return hipSuccess;
}

int32_t next_pow2(int64_t v) {
    int32_t p = 1;
    while (p < v && p < (1 << 30)) p <<= 1;
    return p;
}

// rows per wave of the evaluation kernel: the panel size depends on the row
// count only (so each LP's sums are independent of the batch), with at most
// 2048 panels per side
int32_t eval_rows_per_wave(int32_t rows) {
    int32_t pw = 4;
    while ((int64_t)(rows + 4 * pw - 1) / (4 * pw) > 2048) pw *= 2;
    return pw;
}

}  // namespace

struct Tile {
    int lanes = 64;     // lanes per row group
    int vec = 1;        // consecutive LPs per lane
    int blocks = 0;     // workgroup cap of the launch (0: one wave per row group)
};

constexpr int32_t DEFAULT_MAX_BLOCKS = 16384;
// narrow storage: strides for at most 16, 4, 2, 1 live LPs, and the smallest
// blocks worth the copy
constexpr int32_t NARROW_LD = 16;
constexpr int32_t TINY_LD = 4;
constexpr double NARROW_MIN_BLOCK_BYTES = 256e6;   // one block pair (x rows + y rows)
// largest matrix whose LPs the persistent tail iterates with one workgroup each
constexpr int64_t TAIL_MAX_NNZ = 65536;
constexpr int64_t RUN_AHEAD_AFTER = 8;      // blocks of a solve before replays run ahead of the host
constexpr double RUN_AHEAD_BYTES = 32e6;    // ... and only while one launch moves less than this

struct pdlpb_ctx {
    std::string err = "no error";
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    pdlpb_options opt{};
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    bool fp32 = false;

    // matrix and base vectors on the device
    int32_t *a_rp = nullptr, *a_ci = nullptr, *t_rp = nullptr, *t_ci = nullptr;
    double *a_v64 = nullptr, *t_v64 = nullptr;
    float *a_v32 = nullptr, *t_v32 = nullptr;
    // ELL heads: the first ew entries of every row (index -1 pads short rows)
    int32_t a_ew = 0, t_ew = 0;
    int32_t *a_eci = nullptr, *t_eci = nullptr;
    double *a_ev64 = nullptr, *t_ev64 = nullptr;
    float *a_ev32 = nullptr, *t_ev32 = nullptr;
    double *c = nullptr, *xl = nullptr, *xu = nullptr, *rl = nullptr, *ru = nullptr;
    int8_t* rcode = nullptr;        // per row: 1 if l = -inf, | 2 if u = +inf

    // host copies used by set_batch (the caller's bounds, before any scaling)
    std::vector<double> h_xl, h_xu;
    // diagonal scaling: the solver works on D_r A D_c (all ones when off)
    bool scaled = false;
    std::vector<double> h_dr, h_dc;
    double *d_dr = nullptr, *d_dc = nullptr;
    double norm_c = 0.0, norm_b = 0.0;
    double eta = 0.0, norm_a = 0.0;

    // batch storage
    int32_t B = 0, ld = 0;
    int32_t n_run0 = 0;             // LPs placed in slots by set_batch (the others never run)
    int32_t live = 0;               // live column count the current launches are shaped for
    Tile tp, td;                    // tile shapes of the primal and dual product kernels
    int wpb = 4;
    int vec_ld = 1;                 // vector width ld is padded for
    // tile shapes chosen by timing, per (live column shape, ld)
    std::vector<std::pair<int64_t, std::pair<Tile, Tile>>> tuned;
    size_t cap_block_bytes = 0;     // bytes of each of the 8 dense blocks per row (ld * element size)
    void* blk[8] = {};              // Xbar, X0, Xt, DX, Y, Y0, Yt, DY (row-major, stride ld)
    // Narrow storage: once at most NARROW_LD columns of a wide batch still run,
    // run_solve copies them into blocks of stride NARROW_LD and works there
    // until it returns (blk and ld point at them meanwhile).
    void* nblk[8] = {};             // the narrow blocks (allocated on first use)
    void* tblk[3][8] = {};          // blocks of stride 4, 2 and 1 for the last few LPs (one set
                                    // per stride: captured graphs keep their pointers)
    void* wblk[8] = {};             // the batch's own blocks while narrow storage is in use
    int32_t wld = 0;                // and their stride
    bool narrow = false;
    size_t cap_res_x = 0, cap_res_y = 0;
    void* res[4] = {};              // Rx, Rxi (B x n), Ry, Ryi (B x m): LP-major results
    // the caller's blocks for x~ and y~ of a batch (pdlpb_set_result_buffers)
    double* ext_x = nullptr;
    double* ext_y = nullptr;
    int32_t ext_cap = 0;            // LPs they hold
    // result block q as the kernels write it and the copies read it
    void* out(int q) const {
        if (!serving && ext_x && q == 0) return ext_x;
        if (!serving && ext_y && q == 2) return ext_y;
        return res[q];
    }
    int32_t cap_slots = 0;          // slot (column) capacity
    int32_t cap_lps = 0;            // LP rows of ctl / rlog
    Slots sl{};                     // per-slot arrays (key, tau, sigma, dval, t_start, lp)
    SlotCtl* ctl = nullptr;         // by LP
    int32_t* rlog = nullptr;        // by LP
    RetireEntry* retire = nullptr;
    MoveEntry* moves = nullptr;
    int32_t* fresh = nullptr;       // restarted slots that stay in place (compaction plan)
    Globals* g = nullptr;
    size_t cap_part = 0;            // doubles in part (x and y) + sums
    double* part = nullptr;
    int32_t pw_x = 4, pw_y = 4, npx = 0, npy = 0;
    size_t cap_stage = 0;
    double* stage = nullptr;        // staging for warm starts and results
    double* pow_buf = nullptr;      // power iteration scratch
    int32_t *a_e8ci = nullptr, *t_e8ci = nullptr;   // persistent tail: first 8 entries of
    double *a_e8v64 = nullptr, *t_e8v64 = nullptr;   //   every row of A and A' (small
    float *a_e8v32 = nullptr, *t_e8v32 = nullptr;    //   matrices only; index -1 pads)
    int64_t lds_max = 0;            // LDS bytes a workgroup may hold on the device
    void* tail_work = nullptr;      // persistent tail: contiguous iterates of each LP
    double* tail_sum = nullptr;     //   and its evaluation chain and panel sums
    int32_t tail_cap = 0;           //   LPs the two buffers hold
    int32_t* h_pinned = nullptr;    // n_active read-back
    // serving: the plan of the last admission's compaction (Globals, then up to
    // max_batch retire entries), read by the next serve_wait
    int32_t* h_adm_pin = nullptr;
    bool adm_report = false;
    // shared start: a batch whose running LPs start from one point with the same
    // step sizes makes its first iteration and evaluation per base LP and per
    // change (kernels launch_sp_*)
    std::vector<uint8_t> h_sp_ok;   // per variable: its column and the rows through it fit the caps
    bool sp_batch = false;          // the batch set runs its first iteration that way
    int32_t sp_ncls = 0, sp_cls_obj = -1, sp_cls_bound = -1, sp_kind[2] = {0, 0};
    double sp_tau[2] = {0.0, 0.0}, sp_sigma[2] = {0.0, 0.0};   // per base LP
    void* sp_vec = nullptr;         // base vectors: x0, y0, then per base LP xt, xbar, dx, yt, yn, dy
    void* sp_side = nullptr;        // per slot: SP_SIDE values where its LP differs
    double* sp_terms = nullptr;     // per base LP: row terms, chain sums, panel sums
    int32_t* sp_map = nullptr;      // live columns after the first compaction
    size_t cap_sp_vec = 0, cap_sp_side = 0, cap_sp_terms = 0, cap_sp_map = 0;   // bytes

    // state
    bool batch_set = false;
    bool solved = false;
    std::vector<SlotCtl> h_ctl;
    std::vector<int32_t> h_rlog;
    std::vector<pdlpb_delta> h_delta;   // the batch's changes, by LP

    // captured blocks of C iterations, one per launch configuration; every
    // argument a captured launch holds by value is in the key or is a pointer
    // into storage that only ensure_storage replaces (and it drops the cache)
    struct GraphKey {
        int32_t live, ld, wpb, narrow;
        int32_t tp_lanes, tp_vec, tp_blocks, td_lanes, td_vec, td_blocks;
        const void* rx;   // result blocks the compactions write (the caller's or the context's)
        const void* ry;
        bool operator==(const GraphKey& o) const {
            return live == o.live && ld == o.ld && wpb == o.wpb && narrow == o.narrow &&
                   tp_lanes == o.tp_lanes && tp_vec == o.tp_vec && tp_blocks == o.tp_blocks &&
                   td_lanes == o.td_lanes && td_vec == o.td_vec && td_blocks == o.td_blocks &&
                   rx == o.rx && ry == o.ry;
        }
    };
    std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
    int64_t graph_captures = 0;     // graphs captured and instantiated over the context's life

    // serving (continuous batching)
    struct Pending {
        int32_t row;          // result row (LP index of the kernels)
        int32_t varkind;
        double dval, w, tol;
        int32_t max_iters;
        int32_t warm;         // PDLPB_WARM_NONE or PDLPB_WARM_BASE
    };
    bool serving = false;
    int32_t res_cap = 0;
    int32_t n_cols = 0;                         // live columns after the last wait
    int32_t t0 = 0;                             // global iteration index of the next block's base
    bool launched = false;
    std::vector<int32_t> free_rows;
    std::vector<int64_t> row_id;                // id held by each result row (-1 free)
    enum : int8_t { ROW_FREE = 0, ROW_QUEUED = 1, ROW_RUNNING = 2, ROW_STOPPED = 3 };
    std::vector<int8_t> row_state;              // where the LP of each result row stands
    std::vector<int8_t> row_settled;            // 1: the LP settled at submission (never on the device)
    std::vector<SlotCtl> settled_ctl;           // its outcome, by row
    int32_t row_hi = 0;                         // rows [0, row_hi) hold every row in use
    hipEvent_t serve_ev = nullptr;              // end of the block in flight
    std::unordered_map<int64_t, int32_t> id_row;
    std::deque<Pending> queue;
    std::deque<int64_t> completed;
    int64_t next_id = 0;
    double* base_x = nullptr;                   // resident warm start (n + m doubles)
    double base_w = 0.0;
    bool have_base = false;
    int32_t* adm_rows = nullptr;                // admission staging (capacity columns)
    SlotCtl* adm_ctl = nullptr;
    std::vector<int32_t> h_adm_rows;
    std::vector<SlotCtl> h_adm_ctl;
    std::vector<SlotKey> h_adm_key;
    std::vector<double> h_adm_tau, h_adm_sigma, h_adm_dval;
    std::vector<int32_t> h_adm_tstart, h_adm_lp;
    std::vector<RetireEntry> h_retire;

    // kernel timing
    bool timing = false;
    int64_t t_counts[5] = {0, 0, 0, 0, 0};
    double t_ms[5] = {0, 0, 0, 0, 0};
    int64_t t_cols[5] = {0, 0, 0, 0, 0};   // live LP columns summed over the timed launches
    int32_t cur_cols = 0;               // live LP columns of the launches being enqueued
    std::vector<int32_t> rec_cols;      // cur_cols at each timed launch (by event pair)
    std::vector<hipEvent_t> ev;
    hipEvent_t cnt_ev[2] = {nullptr, nullptr};   // live counts copied to h_pinned[8 + 4 s]

    int64_t dev_bytes = 0;

    // ------------------------------------------------------------------
    int fail(int code, const std::string& msg) {
        err = msg;
        return code;
    }
    int hip_fail(hipError_t e, const char* what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? PDLPB_ENOMEM : PDLPB_EDEVICE;
    }
    // every live device buffer and its size (the free callback takes the size)
    std::unordered_map<void*, size_t> dev_sizes;
    template <typename P>
    hipError_t alloc(P** p, size_t bytes) {
        if (bytes == 0) bytes = 256;
        void* q = nullptr;
        if (opt.dev_alloc) {
            q = opt.dev_alloc(bytes, opt.alloc_user);
            if (!q) return hipErrorOutOfMemory;
        } else {
            hipError_t e = hipMalloc(&q, bytes);
            if (e != hipSuccess) return e;
        }
        dev_sizes[q] = bytes;
        dev_bytes += (int64_t)bytes;
        *p = static_cast<P*>(q);
        return hipSuccess;
    }
    void free_raw(void* q) {
        auto it = dev_sizes.find(q);
        const size_t bytes = it != dev_sizes.end() ? it->second : 0;
        if (it != dev_sizes.end()) dev_sizes.erase(it);
        dev_bytes -= (int64_t)bytes;
        if (opt.dev_free) {
            // a caller's allocator may hand the memory out again at once: no
            // work of this context may still use it
            if (stream) (void)hipStreamSynchronize(stream);
            opt.dev_free(q, bytes, opt.alloc_user);
        } else {
            (void)hipFree(q);
        }
    }
    template <typename P>
    void release(P*& p, size_t /*bytes*/) {
        if (p) free_raw((void*)p);
        p = nullptr;
    }
    void drop_graph() {
        for (auto& gr : graphs) (void)hipGraphExecDestroy(gr.second);
        graphs.clear();
    }
    GraphKey graph_key() const {
        return GraphKey{live,      ld,       wpb,    narrow ? 1 : 0, tp.lanes, tp.vec,
                        tp.blocks, td.lanes, td.vec, td.blocks,      out(0),   out(2)};
    }
};

#define HIP_TRY(ctx, call)                                    \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return (ctx)->hip_fail(e_, #call); \
    } while (0)

namespace {

void free_all(pdlpb_ctx* x) {
    if (!x) return;
    (void)hipSetDevice(x->device);
    if (x->stream) (void)hipStreamSynchronize(x->stream);
    x->drop_graph();
    for (auto e : x->ev) (void)hipEventDestroy(e);
    x->ev.clear();
    for (auto& e : x->cnt_ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    if (x->serve_ev) (void)hipEventDestroy(x->serve_ev);
    // every device buffer, whichever allocator it came from
    std::vector<void*> live;
    live.reserve(x->dev_sizes.size());
    for (auto& kv : x->dev_sizes) live.push_back(kv.first);
    for (void* p : live) x->free_raw(p);
    if (x->h_pinned) (void)hipHostFree(x->h_pinned);
    if (x->h_adm_pin) (void)hipHostFree(x->h_adm_pin);
    if (x->own_stream && x->stream) (void)hipStreamDestroy(x->stream);
    delete x;
}

// ---- step size: power iteration on A'A (float64, on the device) -------------
// ||A||_2 = sqrt(lambda_max(A'A)); start from a normalised Weyl-sequence vector,
// stop when the eigenvalue estimate changes by at most 1e-14 relative, or after
// 10^4 products.  Estimates are read back 32 iterations at a time.
int compute_opnorm(pdlpb_ctx* x, double* out) {
    const int32_t n = x->n, m = x->m;
    if (x->nnz == 0 || n == 0) {
        *out = 0.0;
        return PDLPB_OK;
    }
    constexpr int CH = 32;
    const size_t need = (size_t)n * 2 + (size_t)m + 1024 + CH;
    HIP_TRY(x, x->alloc(&x->pow_buf, need * sizeof(double)));
    double* v = x->pow_buf;
    double* w = v + n;
    double* tmp = w + n;
    double* part = tmp + m;
    double* lam2 = part + 1024;   // CH estimates of lambda^2
    {   // start vector v_j = 1 + frac(j g), g = (sqrt(5)-1)/2, normalised; a constant
        // vector is in the null space of matrices whose rows sum to zero
        std::vector<double> hv(n);
        double s2 = 0.0;
        for (int32_t j = 0; j < n; ++j) {
            const double t = (double)j * 0.6180339887498949;
            hv[j] = 1.0 + (t - std::floor(t));
            s2 += hv[j] * hv[j];
        }
        const double inv = 1.0 / std::sqrt(s2);
        for (double& e : hv) e *= inv;
        HIP_TRY(x, hipMemcpyAsync(v, hv.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                                  x->stream));
        HIP_TRY(x, hipStreamSynchronize(x->stream));
    }
    double lam_old = 0.0;
    double lam = 0.0;
    std::vector<double> h(CH);
    for (int it0 = 0; it0 < 10000; it0 += CH) {
        for (int j = 0; j < CH; ++j) {
            HIP_TRY(x, launch_spmv(x->a_rp, x->a_ci, x->a_v64, m, v, tmp, x->stream));
            HIP_TRY(x, launch_spmv(x->t_rp, x->t_ci, x->t_v64, n, tmp, w, x->stream));
            HIP_TRY(x, launch_norm2sq(w, n, part, lam2 + j, x->stream));
            HIP_TRY(x, launch_scale(w, n, lam2 + j, x->stream));
            std::swap(v, w);
        }
        HIP_TRY(x, hipMemcpyAsync(h.data(), lam2, CH * sizeof(double), hipMemcpyDeviceToHost,
                                  x->stream));
        HIP_TRY(x, hipStreamSynchronize(x->stream));
        for (int j = 0; j < CH && it0 + j < 10000; ++j) {
            lam = std::sqrt(h[j]);
            if (lam == 0.0) {
                *out = 0.0;
                return PDLPB_OK;
            }
            if (std::fabs(lam - lam_old) <= 1e-14 * lam) {
                *out = std::sqrt(lam);
                return PDLPB_OK;
            }
            lam_old = lam;
        }
    }
    *out = std::sqrt(lam);
    return PDLPB_OK;
}

// default tile for `ncols` live columns: a row group covers W = lanes * vec
// consecutive slots with W = 64 (fewer when the batch is narrower), 2 FP64 or
// 4 FP32 slots per lane once the batch is that wide -- the fastest shape of
// the 200k x 500k sweeps at B = 64 ... 512 in both precisions; vec never
// exceeds the width ld was padded for
Tile heuristic_tile(const pdlpb_ctx* x, int32_t ncols) {
    if (x->narrow && x->ld <= TINY_LD) {
        // blocks of stride 4, 2 or 1: one lane per row covers every column
        Tile t;
        t.lanes = 1;
        t.vec = x->ld;
        t.blocks = x->opt.max_blocks > 0 ? x->opt.max_blocks : DEFAULT_MAX_BLOCKS;
        return t;
    }
    const int32_t w = std::min<int32_t>(64, next_pow2(ncols > 0 ? ncols : 1));
    int vec = w >= 64 ? (x->fp32 ? 4 : 2) : 1;
    if (x->opt.tile_vec > 0) vec = x->opt.tile_vec;
    if (vec > x->vec_ld) vec = x->vec_ld;
    // at least 8 lanes per row group: a narrow batch (few live LPs) still spreads
    // its rows over many waves (the idle lanes return at once), which is what
    // keeps the latency-bound iterations of a shrinking batch short
    int lanes = std::max(8, (int)(w / vec));
    if (lanes > 64) lanes = 64;
    if (x->opt.tile_lanes > 0) lanes = x->opt.tile_lanes;
    Tile t;
    t.lanes = lanes;
    t.vec = vec;
    t.blocks = x->opt.max_blocks > 0 ? x->opt.max_blocks : DEFAULT_MAX_BLOCKS;
    return t;
}

void choose_tile(pdlpb_ctx* x, int32_t ncols) {
    x->tp = x->td = heuristic_tile(x, ncols);
    x->wpb = 4;
}

// compulsory bytes of one primal launch at `ncols` columns (the size at which
// timing tile shapes on the live solve pays for itself)
double launch_bytes(const pdlpb_ctx* x, int32_t ncols) {
    const double s = x->fp32 ? 4.0 : 8.0;
    return (double)x->nnz * (s + 4) + s * ncols * ((double)x->m + 3.0 * x->n);
}

// tile shapes worth timing: widths 16..256 (not beyond the next power of two
// above the live columns), every vector width the padding allows
std::vector<Tile> tile_candidates(const pdlpb_ctx* x, int32_t ncols) {
    std::vector<Tile> out;
    const int32_t wmax = std::min<int32_t>(256, next_pow2(ncols));
    for (int vec = 1; vec <= x->vec_ld; vec *= 2)
        for (int32_t w = 16; w <= wmax; w *= 2) {
            const int lanes = w / vec;
            if (lanes < 1 || lanes > 64) continue;
            Tile t;
            t.lanes = lanes;
            t.vec = vec;
            t.blocks = x->opt.max_blocks > 0 ? x->opt.max_blocks : DEFAULT_MAX_BLOCKS;
            out.push_back(t);
        }
    return out;
}

// launch shape for a live column count: the next power of two (at most B), so
// a shrinking batch is re-captured at most log2(B) + 1 times per solve
int32_t shape_cols(const pdlpb_ctx* x, int32_t live) {
    int32_t c = next_pow2(live > 0 ? live : 1);
    return c < x->B ? c : x->B;
}

template <typename T>
StepArgs<T> step_args(pdlpb_ctx* x, bool primal, int32_t it, int32_t eval, int32_t admit = 0) {
    StepArgs<T> a{};
    T* const* b = reinterpret_cast<T* const*>(x->blk);
    const T* av = nullptr;
    if constexpr (sizeof(T) == 8) av = reinterpret_cast<const T*>(primal ? x->t_v64 : x->a_v64);
    else av = reinterpret_cast<const T*>(primal ? x->t_v32 : x->a_v32);
    a.rp = primal ? x->t_rp : x->a_rp;
    a.ci = primal ? x->t_ci : x->a_ci;
    a.av = av;
    a.ew = primal ? x->t_ew : x->a_ew;
    a.eci = primal ? x->t_eci : x->a_eci;
    if constexpr (sizeof(T) == 8) a.ev = reinterpret_cast<const T*>(primal ? x->t_ev64 : x->a_ev64);
    else a.ev = reinterpret_cast<const T*>(primal ? x->t_ev32 : x->a_ev32);
    a.rows = primal ? x->n : x->m;
    a.ld = x->ld;
    a.ncols = x->live;
    a.wpb = x->wpb;
    a.max_blocks = primal ? x->tp.blocks : x->td.blocks;
    if (primal) {
        a.G = b[4];   // Y
        a.Z = b[0]; a.Z0 = b[1]; a.Zt = b[2]; a.DZ = b[3];
        a.c = x->c; a.lo = x->xl; a.hi = x->xu;
    } else {
        a.G = b[0];   // Xbar
        a.Z = b[4]; a.Z0 = b[5]; a.Zt = b[6]; a.DZ = b[7];
        a.c = nullptr; a.lo = x->rl; a.hi = x->ru;
    }
    a.sl = x->sl;
    a.g = x->g;
    a.it = it;
    a.eval = eval;
    a.admit = admit;
    return a;
}

template <typename T>
EvalArgs<T> eval_args(pdlpb_ctx* x, int32_t it, int32_t full) {
    EvalArgs<T> a{};
    a.it = it;
    a.full = full;
    T* const* b = reinterpret_cast<T* const*>(x->blk);
    a.n = x->n; a.m = x->m; a.ld = x->ld; a.ncols = x->live;
    a.a_rp = x->a_rp; a.a_ci = x->a_ci;
    a.t_rp = x->t_rp; a.t_ci = x->t_ci;
    if constexpr (sizeof(T) == 8) {
        a.a_v = reinterpret_cast<const T*>(x->a_v64);
        a.t_v = reinterpret_cast<const T*>(x->t_v64);
    } else {
        a.a_v = reinterpret_cast<const T*>(x->a_v32);
        a.t_v = reinterpret_cast<const T*>(x->t_v32);
    }
    a.Xt = b[2]; a.DX = b[3]; a.X0 = b[1];
    a.Yt = b[6]; a.DY = b[7]; a.Y0 = b[5];
    a.c = x->c; a.xl = x->xl; a.xu = x->xu; a.rl = x->rl; a.ru = x->ru;
    a.rcode = x->rcode;
    a.sl = x->sl;
    a.g = x->g;
    a.pw_x = x->pw_x; a.pw_y = x->pw_y; a.npx = x->npx; a.npy = x->npy;
    a.part_x = x->part;
    a.part_y = x->part + (size_t)x->npx * NTERM * x->ld;
    return a;
}

ControlArgs control_args(pdlpb_ctx* x, int32_t it, int32_t full, int32_t advance,
                         int32_t admit = 0) {
    ControlArgs a{};
    a.ncols = x->live; a.ld = x->ld; a.npx = x->npx; a.npy = x->npy;
    a.part_x = x->part;
    a.part_y = x->part + (size_t)x->npx * NTERM * x->ld;
    a.sums = x->part + (size_t)(x->npx + x->npy) * NTERM * x->ld;
    a.sl = x->sl; a.ctl = x->ctl; a.rlog = x->rlog;
    a.retire = x->retire; a.moves = x->moves; a.fresh = x->fresh; a.g = x->g;
    a.it = it; a.full = full; a.advance = advance; a.block = x->opt.eval_every;
    a.batch_avg = x->opt.restart_scope == PDLPB_RESTART_BATCH_AVG;
    a.pw_literal = x->opt.pw_ratio == 1;
    a.beta_s = x->opt.beta_sufficient; a.beta_n = x->opt.beta_necessary;
    a.beta_a = x->opt.beta_artificial; a.theta = x->opt.theta; a.cross_sign = x->opt.cross_sign;
    a.infeas_tol = x->opt.infeas_tol;   // < 0: the stopping tolerance (resolved on the device)
    a.dual_tol = x->opt.dual_tol;       // < 0: the stopping tolerance (resolved on the device)
    a.admit = admit;
    return a;
}

// event pair index for a timed launch
int timed_begin(pdlpb_ctx* x, int kind, std::vector<std::pair<int, int>>& rec) {
    const int idx = (int)rec.size();
    while ((int)x->ev.size() < 2 * (idx + 1)) {
        hipEvent_t e;
        // timing only: no system-scope fence, so the events neither flush the
        // caches nor slow the launches they bracket
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
        x->ev.push_back(e);
    }
    rec.push_back({kind, idx});
    if ((int)x->rec_cols.size() <= idx) x->rec_cols.resize(idx + 1);
    x->rec_cols[idx] = x->cur_cols;
    (void)hipEventRecord(x->ev[2 * idx], x->stream);
    return idx;
}

template <typename T>
int enqueue_iteration(pdlpb_ctx* x, int32_t it, int32_t eval,
                      std::vector<std::pair<int, int>>* rec, int32_t admit = 0) {
    StepArgs<T> p = step_args<T>(x, true, it, eval, admit);
    StepArgs<T> d = step_args<T>(x, false, it, eval, admit);
    int idx = -1;
    if (rec) idx = timed_begin(x, 0, *rec);
    HIP_TRY(x, launch_primal<T>(p, x->tp.lanes, x->tp.vec, x->stream));
    if (rec && idx >= 0) (void)hipEventRecord(x->ev[2 * idx + 1], x->stream);
    if (rec) idx = timed_begin(x, 1, *rec);
    HIP_TRY(x, launch_dual<T>(d, x->td.lanes, x->td.vec, x->stream));
    if (rec && idx >= 0) (void)hipEventRecord(x->ev[2 * idx + 1], x->stream);
    return PDLPB_OK;
}

template <typename T>
int enqueue_evaluation(pdlpb_ctx* x, int32_t it, int32_t full, int32_t advance,
                       std::vector<std::pair<int, int>>* rec, int32_t admit = 0,
                       int32_t stop = 0) {
    // a stopping test alone needs the sums of every running LP, as a full evaluation
    // does, but only the terms of the stopping measures
    EvalArgs<T> e = eval_args<T>(x, it, full || stop);
    e.kkt_only = stop && !full;
    ControlArgs c = control_args(x, it, full, advance, admit);
    c.stop_only = stop;
    c.admit_plan = admit;
    int idx = -1;
    if (rec) idx = timed_begin(x, 2, *rec);
    HIP_TRY(x, launch_eval<T>(e, x->stream));
    if (rec && idx >= 0) (void)hipEventRecord(x->ev[2 * idx + 1], x->stream);
    if (rec) idx = timed_begin(x, 3, *rec);
    HIP_TRY(x, launch_reduce(c, x->stream));
    HIP_TRY(x, launch_control(c, x->stream));
    if (full || stop) {
        T* const* b = reinterpret_cast<T* const*>(x->blk);
        T* const r[4] = {static_cast<T*>(x->out(0)), static_cast<T*>(x->out(1)),
                         static_cast<T*>(x->out(2)), static_cast<T*>(x->out(3))};
        HIP_TRY(x, launch_compact<T>(x->n, x->m, x->ld, x->live, b, r, x->retire, x->moves,
                                     x->fresh, x->sl, x->g, x->stream));
    }
    if (rec && idx >= 0) (void)hipEventRecord(x->ev[2 * idx + 1], x->stream);
    return PDLPB_OK;
}

// Interval S of the stopping tests between full evaluations (option
// stop_every), 0 when they are off: per-LP restart scope and batches only.
// S >= 2 divides C, so a stopping test never falls on the first iteration of a
// block (the fresh-cycle evaluation) or on its last (the full one).
int32_t stop_interval(const pdlpb_ctx* x) {
    const int32_t S = x->opt.stop_every, C = x->opt.eval_every;
    if (S <= 0 || S >= C || x->serving || x->opt.restart_scope != PDLPB_RESTART_PER_LP) return 0;
    return S;
}
bool stop_at(const pdlpb_ctx* x, int32_t it) {
    const int32_t S = stop_interval(x);
    return S > 0 && it % S == 0 && it != x->opt.eval_every;
}

int read_counts(pdlpb_ctx* x, int32_t* n_active, int32_t* n_cols);

// one block of C iterations: t = t0+1 .. t0+C; residual of fresh cycles at the
// first, stopping tests every S, full evaluation (KKT, restarts) at the last
template <typename T>
int enqueue_epoch(pdlpb_ctx* x, std::vector<std::pair<int, int>>* rec) {
    const int32_t C = x->opt.eval_every;
    for (int32_t it = 1; it <= C; ++it) {
        // z~ stored by every LP before the full evaluation and the stopping
        // tests, by fresh cycles before the first
        const bool stop = stop_at(x, it);
        const int32_t ev = (it == C || stop) ? 2 : (it == 1 ? 1 : 0);
        int rc = enqueue_iteration<T>(x, it, ev, rec);
        if (rc) return rc;
        if (it == C) {
            rc = enqueue_evaluation<T>(x, it, 1, 1, rec);
        } else if (stop) {
            rc = enqueue_evaluation<T>(x, it, 0, 0, rec, 0, 1);
            // timed launches record the live columns they run on, and after a
            // stopping test the device may hold fewer (eager timing only: the
            // host waits for the count; a captured block never does)
            if (!rc && rec) {
                int32_t n_active = 0, n_cols = 0;
                rc = read_counts(x, &n_active, &n_cols);
                if (!rc) x->cur_cols = n_cols;
            }
        } else if (it == 1) {
            rc = enqueue_evaluation<T>(x, it, 0, 0, rec);
        }
        if (rc) return rc;
    }
    return PDLPB_OK;
}

// Launch one block of C iterations as a captured graph: the graph of the
// current launch configuration is reused across batches and serving rounds,
// and captured on first use.  The cache is bounded; past the bound it starts
// over.
constexpr size_t MAX_GRAPHS = 64;

template <typename T>
int replay_epoch(pdlpb_ctx* x) {
    const pdlpb_ctx::GraphKey key = x->graph_key();
    hipGraphExec_t exec = nullptr;
    for (auto& gr : x->graphs)
        if (gr.first == key) exec = gr.second;
    if (!exec) {
        if (x->graphs.size() >= MAX_GRAPHS) {
            // a replay of another graph may still be queued: graphs are only
            // destroyed once the stream has drained
            HIP_TRY(x, hipStreamSynchronize(x->stream));
            x->drop_graph();
        }
        hipGraph_t gr = nullptr;
        HIP_TRY(x, hipStreamBeginCapture(x->stream, hipStreamCaptureModeThreadLocal));
        int r2 = enqueue_epoch<T>(x, nullptr);
        hipError_t e = hipStreamEndCapture(x->stream, &gr);
        if (r2) {
            if (gr) (void)hipGraphDestroy(gr);
            return r2;
        }
        if (e != hipSuccess) return x->hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return x->hip_fail(e, "hipGraphInstantiate");
        x->graphs.push_back({key, exec});
        x->graph_captures += 1;
    }
    HIP_TRY(x, hipGraphLaunch(exec, x->stream));
    return PDLPB_OK;
}

// One block of C iterations that also times tile shapes: the iterations
// between the two evaluations cycle through the candidates, every product
// launch bracketed by events; the fastest shape is kept per kernel.  All
// shapes produce the same bits, so the solve itself is unaffected.
template <typename T>
int tune_epoch(pdlpb_ctx* x) {
    const std::vector<Tile> cand = tile_candidates(x, x->live);
    const int32_t C = x->opt.eval_every;
    const int nc = (int)cand.size();
    std::vector<double> ms(2 * nc, 0.0);
    std::vector<int> cnt(2 * nc, 0);
    std::vector<std::pair<int, int>> rec;   // (candidate * 2 + kernel, event pair)
    const Tile keep_p = x->tp, keep_d = x->td;
    for (int32_t it = 1; it <= C; ++it) {
        const bool stop = stop_at(x, it);
        const bool ev = (it == 1 || it == C || stop);
        int c = -1;
        if (!ev && nc > 0) {
            c = (it - 2) % nc;
            x->tp = x->td = cand[c];
        } else {
            x->tp = keep_p;
            x->td = keep_d;
        }
        const int32_t lev = (it == C || stop) ? 2 : (it == 1 ? 1 : 0);
        StepArgs<T> p = step_args<T>(x, true, it, lev);
        StepArgs<T> d = step_args<T>(x, false, it, lev);
        for (int kern = 0; kern < 2; ++kern) {
            int idx = -1;
            if (c >= 0) idx = timed_begin(x, c * 2 + kern, rec);
            if (kern == 0) HIP_TRY(x, launch_primal<T>(p, x->tp.lanes, x->tp.vec, x->stream));
            else HIP_TRY(x, launch_dual<T>(d, x->td.lanes, x->td.vec, x->stream));
            if (idx >= 0) (void)hipEventRecord(x->ev[2 * idx + 1], x->stream);
        }
        int rc = PDLPB_OK;
        if (it == C) rc = enqueue_evaluation<T>(x, it, 1, 1, nullptr);
        else if (stop) rc = enqueue_evaluation<T>(x, it, 0, 0, nullptr, 0, 1);
        else if (it == 1) rc = enqueue_evaluation<T>(x, it, 0, 0, nullptr);
        if (rc) return rc;
    }
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    // the first sample of each candidate warms caches; average the rest
    std::vector<int> seen(2 * nc, 0);
    for (auto& r : rec) {
        float e = 0.f;
        if (hipEventElapsedTime(&e, x->ev[2 * r.second], x->ev[2 * r.second + 1]) != hipSuccess)
            continue;
        if (seen[r.first]++ == 0) continue;
        ms[r.first] += e;
        cnt[r.first] += 1;
    }
    int bp = -1, bd = -1;
    for (int c = 0; c < nc; ++c) {
        if (cnt[2 * c] && (bp < 0 || ms[2 * c] / cnt[2 * c] < ms[2 * bp] / cnt[2 * bp])) bp = c;
        if (cnt[2 * c + 1] &&
            (bd < 0 || ms[2 * c + 1] / cnt[2 * c + 1] < ms[2 * bd + 1] / cnt[2 * bd + 1]))
            bd = c;
    }
    x->tp = bp >= 0 ? cand[bp] : keep_p;
    x->td = bd >= 0 ? cand[bd] : keep_d;
    x->tuned.push_back({(int64_t)x->live | ((int64_t)x->ld << 32), {x->tp, x->td}});
    return PDLPB_OK;
}

// read the running count and the live column count back to the host
// Queue a copy of the live counts into pinned slot s (0 or 1) and mark it;
// wait_counts reads them once the copy has landed.
int enqueue_counts(pdlpb_ctx* x, int s) {
    if (!x->cnt_ev[s])
        HIP_TRY(x, hipEventCreateWithFlags(&x->cnt_ev[s], hipEventDisableTiming));
    HIP_TRY(x, hipMemcpyAsync(x->h_pinned + 8 + 4 * s, x->g, 4 * sizeof(int32_t),
                              hipMemcpyDeviceToHost, x->stream));
    HIP_TRY(x, hipEventRecord(x->cnt_ev[s], x->stream));
    return PDLPB_OK;
}

int wait_counts(pdlpb_ctx* x, int s, int32_t* n_active, int32_t* n_cols) {
    HIP_TRY(x, hipEventSynchronize(x->cnt_ev[s]));
    *n_active = x->h_pinned[8 + 4 * s + 1];   // Globals::n_active
    *n_cols = x->h_pinned[8 + 4 * s + 3];     // Globals::n_cols
    return PDLPB_OK;
}

int read_counts(pdlpb_ctx* x, int32_t* n_active, int32_t* n_cols) {
    HIP_TRY(x, hipMemcpyAsync(x->h_pinned, x->g, 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                              x->stream));
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    *n_active = x->h_pinned[1];   // Globals::n_active
    *n_cols = x->h_pinned[3];     // Globals::n_cols
    return PDLPB_OK;
}

// LDS the tail kernel needs beyond its static arrays: Xbar and Y of its LP
size_t tail_dyn_lds(const pdlpb_ctx* x) {
    return ((size_t)x->n + (size_t)x->m) * (x->fp32 ? sizeof(float) : sizeof(double));
}

bool tail_applies(const pdlpb_ctx* x, int32_t n_cols) {
    return x->opt.tail_cols > 0 && n_cols > 0 && n_cols <= x->opt.tail_cols &&
           x->nnz <= TAIL_MAX_NNZ && x->opt.restart_scope == PDLPB_RESTART_PER_LP &&
           !x->serving && x->a_e8ci && (int64_t)(tail_dyn_lds(x) + TAIL_STATIC_LDS) <= x->lds_max;
}

// Finish the running LPs of slots [0, n_cols) with the persistent tail kernel
// (one workgroup each), from the next block base on the device.
template <typename T>
int run_tail(pdlpb_ctx* x, int32_t n_cols, std::vector<std::pair<int, int>>* rec) {
    const size_t esz = sizeof(T);
    if (n_cols > x->tail_cap) {
        x->release(x->tail_work, 0);
        x->release(x->tail_sum, 0);
        x->tail_cap = 0;
        const int32_t cap = x->opt.tail_cols;
        HIP_TRY(x, x->alloc(&x->tail_work, (size_t)cap * (4 * (size_t)x->n + 4 * (size_t)x->m) * esz));
        HIP_TRY(x, x->alloc(&x->tail_sum, (size_t)cap * tail_sum_doubles(x->npx, x->npy) * sizeof(double)));
        x->tail_cap = cap;
    }
    TailArgs<T> a{};
    a.n = x->n; a.m = x->m; a.ld = x->ld; a.C = x->opt.eval_every; a.ncols = n_cols;
    a.S = stop_interval(x);
    a.a_rp = x->a_rp; a.a_ci = x->a_ci; a.t_rp = x->t_rp; a.t_ci = x->t_ci;
    if constexpr (sizeof(T) == 8) {
        a.a_v = reinterpret_cast<const T*>(x->a_v64);
        a.t_v = reinterpret_cast<const T*>(x->t_v64);
        a.a_e8v = reinterpret_cast<const T*>(x->a_e8v64);
        a.t_e8v = reinterpret_cast<const T*>(x->t_e8v64);
    } else {
        a.a_v = reinterpret_cast<const T*>(x->a_v32);
        a.t_v = reinterpret_cast<const T*>(x->t_v32);
        a.a_e8v = reinterpret_cast<const T*>(x->a_e8v32);
        a.t_e8v = reinterpret_cast<const T*>(x->t_e8v32);
    }
    a.a_e8ci = x->a_e8ci;
    a.t_e8ci = x->t_e8ci;
    for (int b = 0; b < 8; ++b) a.blk[b] = static_cast<T*>(x->blk[b]);
    for (int b = 0; b < 4; ++b) a.res[b] = static_cast<T*>(x->out(b));
    a.c = x->c; a.xl = x->xl; a.xu = x->xu; a.rl = x->rl; a.ru = x->ru;
    a.sl = x->sl; a.ctl = x->ctl; a.rlog = x->rlog; a.g = x->g;
    a.ca = control_args(x, 0, 1, 0);
    a.pw_x = x->pw_x; a.pw_y = x->pw_y; a.npx = x->npx; a.npy = x->npy;
    a.work = static_cast<T*>(x->tail_work);
    a.wsum = x->tail_sum;
    int idx = -1;
    if (rec) {
        x->cur_cols = n_cols;
        idx = timed_begin(x, 4, *rec);
    }
    HIP_TRY(x, launch_tail<T>(a, tail_dyn_lds(x), x->stream));
    if (rec && idx >= 0) (void)hipEventRecord(x->ev[2 * idx + 1], x->stream);
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    return PDLPB_OK;
}

// Narrow storage.  In the batch's blocks the live columns of a row sit at
// stride ld, so once few LPs run every gathered segment and every streamed row
// lies in its own ld-wide row: at 200k x 500k, 8 running LPs cost 67 / 55 us
// per primal / dual launch in blocks of stride 512 and 48 / 46 us in blocks of
// stride 8.  Once at most NARROW_LD columns of a batch at least four times as
// wide still run, and its blocks exceed the last-level cache, run_solve copies
// those columns into blocks of stride NARROW_LD and works there until it
// returns; once at most 4, 2 or 1 run, into blocks of that stride, where one
// lane takes a whole row (all its columns) and a wave 64 rows: a lone LP's
// vectors are then contiguous, and the one the products gather stays in the
// L2 cache.  Every kernel takes the stride as an argument and every LP's
// arithmetic is independent of it, so results do not change.

// stride the live columns move to now (0: they stay)
int32_t narrow_target(const pdlpb_ctx* x, int32_t n_cols) {
    if (x->serving || n_cols <= 0 || n_cols > NARROW_LD) return 0;
    // blocks that the caches hold gain nothing from the copy
    const double esz = x->fp32 ? 4.0 : 8.0;
    const double row_bytes = ((double)x->n + (double)x->m) * esz;
    const int32_t wide = x->narrow ? x->wld : x->ld;
    if (wide < 4 * NARROW_LD || row_bytes * wide < NARROW_MIN_BLOCK_BYTES) return 0;
    // fixed tile shapes (options, pdlpb_set_tile) keep to the stride-16 blocks
    const bool fixed = x->opt.tile_lanes > 0 || x->opt.tile_vec > 0;
    int32_t want = NARROW_LD;
    if (!fixed) want = n_cols <= 1 ? 1 : n_cols <= 2 ? 2 : n_cols <= TINY_LD ? TINY_LD : NARROW_LD;
    if (want == NARROW_LD && NARROW_LD % x->vec_ld != 0) return 0;
    return want < x->ld ? want : 0;
}

int enter_narrow(pdlpb_ctx* x, int32_t ld) {
    const size_t esz = x->fp32 ? sizeof(float) : sizeof(double);
    void** dst = ld == NARROW_LD ? x->nblk : x->tblk[ld == TINY_LD ? 0 : ld == 2 ? 1 : 2];
    for (int q = 0; q < 8; ++q) {
        const int32_t rows = q < 4 ? x->n : x->m;
        if (!dst[q]) HIP_TRY(x, x->alloc(&dst[q], (size_t)rows * ld * esz));
        if (rows > 0)
            HIP_TRY(x, hipMemcpy2DAsync(dst[q], (size_t)ld * esz, x->blk[q], (size_t)x->ld * esz,
                                        (size_t)ld * esz, (size_t)rows, hipMemcpyDeviceToDevice,
                                        x->stream));
    }
    if (!x->narrow) {
        for (int q = 0; q < 8; ++q) x->wblk[q] = x->blk[q];
        x->wld = x->ld;
    }
    for (int q = 0; q < 8; ++q) x->blk[q] = dst[q];
    x->ld = ld;
    x->narrow = true;
    return PDLPB_OK;
}

void leave_narrow(pdlpb_ctx* x) {
    if (!x->narrow) return;
    for (int q = 0; q < 8; ++q) x->blk[q] = x->wblk[q];
    x->ld = x->wld;
    x->narrow = false;
}

void free_narrow(pdlpb_ctx* x) {
    leave_narrow(x);
    for (int q = 0; q < 8; ++q) {
        x->release(x->nblk[q], 0);
        for (int k = 0; k < 3; ++k) x->release(x->tblk[k][q], 0);
    }
}

// ---- shared start ------------------------------------------------------------
// Automatic choice: blocks of the batch at least this large.  Below, the
// full-width start costs little, while an LP's change may reach a tenth of the
// evaluation panels (20k x 50k, 8 nonzeros per column), each then recomputed
// for that LP alone.
constexpr double SP_AUTO_BYTES = 256e6;

int ensure_bytes(pdlpb_ctx* x, void** p, size_t* cap, size_t bytes) {
    if (bytes <= *cap && *p) return PDLPB_OK;
    x->release(*p, *cap);
    *cap = 0;
    HIP_TRY(x, x->alloc(p, bytes));
    *cap = bytes;
    return PDLPB_OK;
}

void free_shared_start(pdlpb_ctx* x) {
    x->sp_batch = false;
    x->release(x->sp_vec, 0);
    x->release(x->sp_side, 0);
    x->release(x->sp_terms, 0);
    x->release(x->sp_map, 0);
    x->cap_sp_vec = x->cap_sp_side = x->cap_sp_terms = x->cap_sp_map = 0;
}

// Whether the batch just placed in slots makes its first iteration and
// evaluation through the shared start (option shared_start): every running LP
// starts from the shared warm point (or zero), the LPs of one base LP share
// their step sizes, and every change is of a variable within the caps.  Sets
// the base LPs and sizes the buffers when it does.
int plan_shared_start(pdlpb_ctx* x, int32_t warm_mode, const std::vector<SlotKey>& key,
                      const std::vector<double>& tau, const std::vector<double>& sigma) {
    x->sp_batch = false;
    const int32_t nr = (int32_t)key.size();
    if (x->opt.shared_start < 0 || nr == 0) return PDLPB_OK;
    if (warm_mode != PDLPB_WARM_NONE && warm_mode != PDLPB_WARM_SHARED) return PDLPB_OK;
    const size_t esz = x->fp32 ? sizeof(float) : sizeof(double);
    const size_t rows = (size_t)x->n + x->m;
    if (x->opt.shared_start == 0 && (double)rows * nr * esz < SP_AUTO_BYTES) return PDLPB_OK;
    // first LP of each base LP (0: bound changes and the base LP, 1: objective changes)
    int32_t first[2] = {-1, -1};
    for (int32_t s = 0; s < nr; ++s) {
        const int32_t v = key[s].varkind & VAR_MASK;
        if (v != VAR_NONE && !x->h_sp_ok[v]) return PDLPB_OK;
        const int f = ((uint32_t)key[s].varkind >> 28) == (uint32_t)PDLPB_OBJ_UNIT ? 1 : 0;
        if (first[f] < 0) first[f] = s;
        if (tau[s] != tau[first[f]] || sigma[s] != sigma[first[f]]) return PDLPB_OK;
    }
    x->sp_ncls = 0;
    x->sp_cls_obj = x->sp_cls_bound = -1;
    for (int f = 0; f < 2; ++f) {
        if (first[f] < 0) continue;
        const int32_t K = x->sp_ncls++;
        if (f == 0) x->sp_cls_bound = K;
        else x->sp_cls_obj = K;
        x->sp_kind[K] = f == 0 ? PDLPB_BASE : PDLPB_OBJ_UNIT;
        x->sp_tau[K] = tau[first[f]];
        x->sp_sigma[K] = sigma[first[f]];
    }
    const size_t K = (size_t)x->sp_ncls;
    const size_t panels = (size_t)x->npx + x->npy;
    int rc = ensure_bytes(x, &x->sp_vec, &x->cap_sp_vec, rows * (1 + 3 * K) * esz);
    if (!rc) rc = ensure_bytes(x, &x->sp_side, &x->cap_sp_side, (size_t)nr * SP_SIDE * esz);
    if (!rc)
        rc = ensure_bytes(x, reinterpret_cast<void**>(&x->sp_terms), &x->cap_sp_terms,
                          K * (rows + panels * 5) * NTERM * sizeof(double));
    if (!rc)
        rc = ensure_bytes(x, reinterpret_cast<void**>(&x->sp_map), &x->cap_sp_map,
                          (size_t)2 * nr * sizeof(int32_t));
    if (rc) return rc;
    x->sp_batch = true;
    return PDLPB_OK;
}

template <typename T>
SharedArgs<T> shared_args(pdlpb_ctx* x, const double* xw = nullptr, const double* yw = nullptr) {
    SharedArgs<T> a{};
    a.n = x->n;
    a.m = x->m;
    a.ld = x->ld;
    a.nslots = x->n_run0;
    a.ncls = x->sp_ncls;
    a.cls_kind[0] = x->sp_kind[0];
    a.cls_kind[1] = x->sp_kind[1];
    a.cls_obj = x->sp_cls_obj;
    a.cls_bound = x->sp_cls_bound;
    a.a_rp = x->a_rp; a.a_ci = x->a_ci;
    a.t_rp = x->t_rp; a.t_ci = x->t_ci;
    if constexpr (sizeof(T) == 8) {
        a.a_v = reinterpret_cast<const T*>(x->a_v64);
        a.t_v = reinterpret_cast<const T*>(x->t_v64);
    } else {
        a.a_v = reinterpret_cast<const T*>(x->a_v32);
        a.t_v = reinterpret_cast<const T*>(x->t_v32);
    }
    a.c = x->c; a.xl = x->xl; a.xu = x->xu; a.rl = x->rl; a.ru = x->ru;
    a.rcode = x->rcode;
    a.xw = xw;
    a.yw = yw;
    for (int K = 0; K < 2; ++K) {
        a.tau[K] = x->sp_tau[K];
        a.sigma[K] = x->sp_sigma[K];
    }
    const size_t n = x->n, m = x->m, K = x->sp_ncls;
    a.x0 = static_cast<T*>(x->sp_vec);
    a.y0 = a.x0 + n;
    a.xt = a.y0 + m;
    a.xbar = a.xt + K * n;
    a.dx = a.xbar + K * n;
    a.yt = a.dx + K * n;
    a.yn = a.yt + K * m;
    a.dy = a.yn + K * m;
    a.side = static_cast<T*>(x->sp_side);
    a.sl = x->sl;
    a.pw_x = x->pw_x; a.pw_y = x->pw_y; a.npx = x->npx; a.npy = x->npy;
    a.rt = x->sp_terms;
    a.bwave = a.rt + K * (n + m) * NTERM;
    a.bpanel = a.bwave + K * ((size_t)x->npx + x->npy) * 4 * NTERM;
    a.part_x = x->part;
    a.part_y = x->part + (size_t)x->npx * NTERM * x->ld;
    a.g = x->g;
    a.retire = x->retire;
    a.moves = x->moves;
    a.map = x->sp_map;
    for (int b = 0; b < 8; ++b) a.blk[b] = static_cast<T*>(x->blk[b]);
    for (int b = 0; b < 4; ++b) a.res[b] = static_cast<T*>(x->out(b));
    return a;
}

// t = 0 of a shared-start batch (its first iteration was made at set_batch):
// the evaluation sums, the control pass (a full evaluation), then the blocks of
// the LPs still running and the results of those that stopped.
template <typename T>
int enqueue_shared_prologue(pdlpb_ctx* x, std::vector<std::pair<int, int>>* rec) {
    const SharedArgs<T> a = shared_args<T>(x);
    const ControlArgs c = control_args(x, 0, 1, 0);
    int idx = -1;
    if (rec) idx = timed_begin(x, 2, *rec);
    HIP_TRY(x, launch_sp_eval<T>(a, x->stream));
    if (rec && idx >= 0) (void)hipEventRecord(x->ev[2 * idx + 1], x->stream);
    if (rec) idx = timed_begin(x, 3, *rec);
    HIP_TRY(x, launch_reduce(c, x->stream));
    HIP_TRY(x, launch_control(c, x->stream));
    HIP_TRY(x, launch_sp_place<T>(a, x->stream));
    if (rec && idx >= 0) (void)hipEventRecord(x->ev[2 * idx + 1], x->stream);
    return PDLPB_OK;
}

template <typename T>
int run_solve(pdlpb_ctx* x, double tol, int32_t max_iters) {
    x->live = shape_cols(x, x->n_run0);
    choose_tile(x, x->live);
    HIP_TRY(x, launch_begin_solve(x->sl, x->ctl, x->n_run0, max_iters, x->g, tol,
                                  x->stream));
    std::vector<std::pair<int, int>> rec;
    std::vector<std::pair<int, int>>* prec = x->timing ? &rec : nullptr;
    auto harvest = [&]() {
        for (auto& r : rec) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, x->ev[2 * r.second], x->ev[2 * r.second + 1]) ==
                hipSuccess) {
                x->t_counts[r.first] += 1;
                x->t_ms[r.first] += ms;
                x->t_cols[r.first] += x->rec_cols[r.second];
            }
        }
        rec.clear();
    };
    // prologue: t = 0 is a full evaluation
    x->cur_cols = x->n_run0;
    int rc = PDLPB_OK;
    if (x->sp_batch) {
        x->sp_batch = false;
        rc = enqueue_shared_prologue<T>(x, prec);
    } else {
        rc = enqueue_iteration<T>(x, 0, 2, prec);
        if (!rc) rc = enqueue_evaluation<T>(x, 0, 1, 0, prec);
    }
    if (rc) return rc;
    int32_t n_active = 0, n_cols = 0;
    rc = read_counts(x, &n_active, &n_cols);
    if (rc) return rc;
    if (prec) harvest();
    const bool use_graphs = x->opt.use_graphs && !x->timing;
    const int64_t max_epochs = (int64_t)max_iters / x->opt.eval_every + 2;
    // Replayed blocks of a long solve run one ahead of the host: block e+1 is
    // queued before the host waits for the counts of block e, so the device
    // does not idle while the host reads them and decides the next launch
    // shape.  A block queued after every LP has stopped launches kernels that
    // find no live column, which costs little only when the launches are small
    // (latency-bound), and pays off only over many blocks.
    bool in_flight = false;   // a block whose counts have not been read
    int in_slot = 0, next_slot = 0;
    int64_t launched = 0;
    // no block outlives the call: other entry points write device state with
    // copies that do not wait for the context's (non-blocking) stream
    struct Drain {
        pdlpb_ctx* x;
        const bool* f;
        ~Drain() {
            if (*f) (void)hipStreamSynchronize(x->stream);
        }
    } drain{x, &in_flight};
    // the batch's own blocks again when the call returns (the work queued on
    // the narrow ones stays ordered before anything later on the stream)
    struct Wide {
        pdlpb_ctx* x;
        ~Wide() { leave_narrow(x); }
    } wide{x};
    for (int64_t ep = 0; n_active > 0; ++ep) {
        if (launched > max_epochs + 1) return x->fail(PDLPB_EDEVICE, "solve did not terminate");
        if (tail_applies(x, n_cols)) {
            if (in_flight) {
                // the counts of the block running ahead decide first
                rc = wait_counts(x, in_slot, &n_active, &n_cols);
                if (rc) return rc;
                in_flight = false;
                continue;
            }
            // the few LPs left run to their stop in one launch
            rc = run_tail<T>(x, n_cols, prec);
            if (rc) return rc;
            if (prec) harvest();
            return PDLPB_OK;
        }
        if (const int32_t nld = narrow_target(x, n_cols)) {
            if (in_flight) {
                rc = wait_counts(x, in_slot, &n_active, &n_cols);
                if (rc) return rc;
                in_flight = false;
                continue;
            }
            rc = enter_narrow(x, nld);
            if (rc) return rc;
            x->live = -1;   // shape the launches (and their graphs) for the new stride
        }
        // shape the launches for the live columns (compaction shrinks them)
        const int32_t shape = shape_cols(x, n_cols);
        x->cur_cols = n_cols;
        bool tune_now = false;
        if (shape != x->live || ep == 0) {
            x->live = shape;
            choose_tile(x, shape);
            const bool fixed = x->opt.tile_lanes > 0 || x->opt.tile_vec > 0;
            if (x->opt.autotune && !fixed && launch_bytes(x, shape) >= 32e6) {
                const int64_t key = (int64_t)shape | ((int64_t)x->ld << 32);
                bool hit = false;
                for (auto& e : x->tuned)
                    if (e.first == key) {
                        x->tp = e.second.first;
                        x->td = e.second.second;
                        hit = true;
                    }
                tune_now = !hit && !x->timing;
            }
        }
        const bool ahead = use_graphs && !tune_now && launched >= RUN_AHEAD_AFTER &&
                           launch_bytes(x, x->live) < RUN_AHEAD_BYTES;
        if (in_flight && !ahead) {
            // a synchronous block follows: read the counts of the block ahead first
            rc = wait_counts(x, in_slot, &n_active, &n_cols);
            if (rc) return rc;
            in_flight = false;
            continue;
        }
        ++launched;
        if (tune_now) {
            rc = tune_epoch<T>(x);
            if (rc) return rc;
        } else if (use_graphs) {
            rc = replay_epoch<T>(x);
            if (rc) return rc;
            if (ahead) {
                rc = enqueue_counts(x, next_slot);
                if (rc) return rc;
                if (in_flight) {
                    rc = wait_counts(x, in_slot, &n_active, &n_cols);
                    if (rc) return rc;
                }
                in_flight = true;
                in_slot = next_slot;
                next_slot ^= 1;
                continue;
            }
        } else {
            rc = enqueue_epoch<T>(x, prec);
            if (rc) return rc;
        }
        rc = read_counts(x, &n_active, &n_cols);
        if (rc) return rc;
        if (prec) harvest();
    }
    return PDLPB_OK;
}

int fetch_state(pdlpb_ctx* x) {
    x->h_ctl.resize(x->B);
    x->h_rlog.resize((size_t)x->B * RESTART_LOG);
    HIP_TRY(x, hipMemcpyAsync(x->h_ctl.data(), x->ctl, sizeof(SlotCtl) * x->B,
                              hipMemcpyDeviceToHost, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->h_rlog.data(), x->rlog, sizeof(int32_t) * RESTART_LOG * x->B,
                              hipMemcpyDeviceToHost, x->stream));
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    return PDLPB_OK;
}

int ensure_stage(pdlpb_ctx* x, size_t doubles) {
    if (doubles <= x->cap_stage) return PDLPB_OK;
    x->release(x->stage, x->cap_stage * sizeof(double));
    x->cap_stage = 0;
    HIP_TRY(x, x->alloc(&x->stage, doubles * sizeof(double)));
    x->cap_stage = doubles;
    return PDLPB_OK;
}

// Copy `count` LPs starting at LP `first` of result block q (0: x~, 1: Halpern x,
// 2: y~, 3: Halpern y; LP-major) into dst as float64.
int copy_results(pdlpb_ctx* x, int q, int32_t first, int32_t count, double* dst, int32_t mem) {
    const int64_t rows = (q < 2) ? x->n : x->m;
    const int64_t cnt = rows * count;
    if (cnt == 0) return PDLPB_OK;
    // results the solve wrote into these very buffers (pdlpb_set_result_buffers)
    if (mem == PDLPB_MEM_DEVICE && !x->fp32 && !x->scaled &&
        dst == static_cast<const double*>(x->out(q)) + (size_t)first * rows)
        return PDLPB_OK;
    const hipMemcpyKind kind = mem == PDLPB_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                        : hipMemcpyDeviceToHost;
    if (x->scaled) {
        // back to the caller's coordinates: x = dc x^, y = dr y^
        const double* d = q < 2 ? x->d_dc : x->d_dr;
        double* buf = dst;
        if (mem != PDLPB_MEM_DEVICE) {
            int rc = ensure_stage(x, (size_t)cnt);
            if (rc) return rc;
            buf = x->stage;
        }
        if (x->fp32) {
            const float* src = static_cast<const float*>(x->out(q)) + (size_t)first * rows;
            HIP_TRY(x, launch_widen(src, cnt, buf, x->stream));
        } else {
            const double* src = static_cast<const double*>(x->out(q)) + (size_t)first * rows;
            HIP_TRY(x, hipMemcpyAsync(buf, src, cnt * sizeof(double), hipMemcpyDeviceToDevice,
                                      x->stream));
        }
        HIP_TRY(x, launch_rescale(buf, d, cnt, (int32_t)rows, 0, x->stream));
        if (buf != dst)
            HIP_TRY(x, hipMemcpyAsync(dst, buf, cnt * sizeof(double), kind, x->stream));
        HIP_TRY(x, hipStreamSynchronize(x->stream));
        return PDLPB_OK;
    }
    if (x->fp32) {
        const float* src = static_cast<const float*>(x->out(q)) + (size_t)first * rows;
        if (mem == PDLPB_MEM_DEVICE) {
            HIP_TRY(x, launch_widen(src, cnt, dst, x->stream));
        } else {
            int rc = ensure_stage(x, (size_t)cnt);
            if (rc) return rc;
            HIP_TRY(x, launch_widen(src, cnt, x->stage, x->stream));
            HIP_TRY(x, hipMemcpyAsync(dst, x->stage, cnt * sizeof(double), kind, x->stream));
        }
    } else {
        const double* src = static_cast<const double*>(x->out(q)) + (size_t)first * rows;
        HIP_TRY(x, hipMemcpyAsync(dst, src, cnt * sizeof(double), kind, x->stream));
    }
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    return PDLPB_OK;
}

// Status of an LP before it iterates: its change may be malformed or cross its bounds.
int32_t lp_status(const pdlpb_ctx* x, const pdlpb_delta& q) {
    if (q.kind == PDLPB_BASE) return PDLPB_STATUS_RUNNING;
    const bool bad_value = std::isnan(q.value) || (q.kind == PDLPB_SET_LO && q.value == INFINITY) ||
                           (q.kind == PDLPB_SET_HI && q.value == -INFINITY) ||
                           (q.kind == PDLPB_OBJ_UNIT && !std::isfinite(q.value));
    if (bad_value) return PDLPB_STATUS_INVALID_INPUT;
    if (q.kind == PDLPB_SET_LO && q.value > x->h_xu[q.var]) return PDLPB_STATUS_INFEASIBLE_BOUNDS;
    if (q.kind == PDLPB_SET_HI && q.value < x->h_xl[q.var]) return PDLPB_STATUS_INFEASIBLE_BOUNDS;
    return PDLPB_STATUS_RUNNING;
}

// Diagonal scaling of A (pdlpb_options.scaling = 1): `iters` Ruiz passes, each
// dividing every row and column of the current D_r A D_c by the square root
// of its infinity norm (both from the same pass's matrix), then one
// Pock-Chambolle pass with alpha = 1 (square roots of the row and column
// 1-norms).  Empty rows and columns keep the factor 1.
void compute_scaling(int32_t m, int32_t n, const int64_t* rp, const int32_t* ci,
                     const double* v, int iters, std::vector<double>& dr,
                     std::vector<double>& dc) {
    dr.assign(m, 1.0);
    dc.assign(n, 1.0);
    std::vector<double> rs(m), cs(n);
    auto scaled = [&](int32_t i, int64_t k) { return std::fabs((dr[i] * v[k]) * dc[ci[k]]); };
    for (int it = 0; it < iters; ++it) {
        std::fill(rs.begin(), rs.end(), 0.0);
        std::fill(cs.begin(), cs.end(), 0.0);
        for (int32_t i = 0; i < m; ++i)
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                const double a = scaled(i, k);
                rs[i] = std::max(rs[i], a);
                cs[ci[k]] = std::max(cs[ci[k]], a);
            }
        for (int32_t i = 0; i < m; ++i)
            if (rs[i] > 0.0) dr[i] = dr[i] * (1.0 / std::sqrt(rs[i]));
        for (int32_t j = 0; j < n; ++j)
            if (cs[j] > 0.0) dc[j] = dc[j] * (1.0 / std::sqrt(cs[j]));
    }
    std::fill(rs.begin(), rs.end(), 0.0);
    std::fill(cs.begin(), cs.end(), 0.0);
    for (int32_t i = 0; i < m; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const double a = scaled(i, k);
            rs[i] += a;
            cs[ci[k]] += a;
        }
    for (int32_t i = 0; i < m; ++i)
        if (rs[i] > 0.0) dr[i] = dr[i] * (1.0 / std::sqrt(rs[i]));
    for (int32_t j = 0; j < n; ++j)
        if (cs[j] > 0.0) dc[j] = dc[j] * (1.0 / std::sqrt(cs[j]));
}

// A change of the caller's LP expressed on the scaled one: a bound on x_var
// becomes value / dc[var], the objective value * e_var becomes value * dc[var].
pdlpb_delta scaled_delta(const pdlpb_ctx* x, const pdlpb_delta& q) {
    pdlpb_delta r = q;
    if (!x->scaled || q.kind == PDLPB_BASE) return r;
    if (q.kind == PDLPB_OBJ_UNIT) r.value = q.value * x->h_dc[q.var];
    else r.value = q.value / x->h_dc[q.var];
    return r;
}

// Initial primal weight without a warm start: ||c_j|| / ||b|| when both exceed 1e-10, else 1.
double default_weight(const pdlpb_ctx* x, const pdlpb_delta& q) {
    const double cn = q.kind == PDLPB_OBJ_UNIT ? std::fabs(q.value) : x->norm_c;
    return (cn > 1e-10 && x->norm_b > 1e-10) ? cn / x->norm_b : 1.0;
}

// Vector width the row stride of a `cols`-column storage is padded for: 4 when
// the launches are large enough to be tuned over every shape, else the width
// the default tile uses.
int32_t vec_for(const pdlpb_ctx* x, int32_t cols) {
    if (x->opt.autotune && x->opt.tile_vec == 0 && launch_bytes(x, cols) >= 32e6) return 4;
    const int32_t w = std::min<int32_t>(64, next_pow2(cols > 0 ? cols : 1));
    int32_t vec = w >= 64 ? (x->fp32 ? 4 : 2) : 1;
    if (x->opt.tile_vec > 0) vec = x->opt.tile_vec;
    return vec;
}
int32_t ld_for(const pdlpb_ctx* x, int32_t cols) {
    const int32_t v = vec_for(x, cols);
    return ((cols + v - 1) / v) * v;
}

// Device storage for `cols` LP columns and `lps` LP result rows (grows, reused
// for smaller requests).  Sets vec_ld and returns the row stride ld.
int ensure_storage(pdlpb_ctx* x, int32_t cols, int32_t lps, int32_t* ld_out) {
    const int32_t n = x->n, m = x->m;
    // pad for 4-wide vectors when the batch is large enough to be tuned
    x->vec_ld = vec_for(x, cols);
    const int32_t ld = ld_for(x, cols);
    const size_t esz = x->fp32 ? sizeof(float) : sizeof(double);
    // blocks 0-3 hold x rows (n), blocks 4-7 y rows (m); capacity is kept as
    // bytes per row so both kinds grow together
    const size_t row_bytes = (size_t)ld * esz;
    if (row_bytes > x->cap_block_bytes) {
        x->drop_graph();
        for (int q = 0; q < 8; ++q)
            x->release(x->blk[q], (size_t)(q < 4 ? n : m) * x->cap_block_bytes);
        x->cap_block_bytes = 0;
        for (int q = 0; q < 8; ++q)
            HIP_TRY(x, x->alloc(&x->blk[q], (size_t)(q < 4 ? n : m) * row_bytes));
        x->cap_block_bytes = row_bytes;
    }
    const size_t rx_bytes = (size_t)lps * n * esz, ry_bytes = (size_t)lps * m * esz;
    if (rx_bytes > x->cap_res_x || ry_bytes > x->cap_res_y) {
        x->drop_graph();
        x->release(x->res[0], x->cap_res_x);
        x->release(x->res[1], x->cap_res_x);
        x->release(x->res[2], x->cap_res_y);
        x->release(x->res[3], x->cap_res_y);
        x->cap_res_x = x->cap_res_y = 0;
        for (int q = 0; q < 2; ++q) HIP_TRY(x, x->alloc(&x->res[q], rx_bytes));
        for (int q = 2; q < 4; ++q) HIP_TRY(x, x->alloc(&x->res[q], ry_bytes));
        x->cap_res_x = rx_bytes;
        x->cap_res_y = ry_bytes;
    }
    if (cols > x->cap_slots) {
        x->drop_graph();
        x->release(x->sl.key, sizeof(SlotKey) * x->cap_slots);
        x->release(x->sl.tau, sizeof(double) * x->cap_slots);
        x->release(x->sl.sigma, sizeof(double) * x->cap_slots);
        x->release(x->sl.dval, sizeof(double) * x->cap_slots);
        x->release(x->sl.t_start, sizeof(int32_t) * x->cap_slots);
        x->release(x->sl.lp, sizeof(int32_t) * x->cap_slots);
        x->release(x->retire, sizeof(RetireEntry) * x->cap_slots);
        x->release(x->moves, sizeof(MoveEntry) * x->cap_slots);
        x->release(x->fresh, sizeof(int32_t) * x->cap_slots);
        x->release(x->adm_rows, sizeof(int32_t) * x->cap_slots);
        x->release(x->adm_ctl, sizeof(SlotCtl) * x->cap_slots);
        x->cap_slots = 0;
        HIP_TRY(x, x->alloc(&x->sl.key, sizeof(SlotKey) * cols));
        HIP_TRY(x, x->alloc(&x->sl.tau, sizeof(double) * cols));
        HIP_TRY(x, x->alloc(&x->sl.sigma, sizeof(double) * cols));
        HIP_TRY(x, x->alloc(&x->sl.dval, sizeof(double) * cols));
        HIP_TRY(x, x->alloc(&x->sl.t_start, sizeof(int32_t) * cols));
        HIP_TRY(x, x->alloc(&x->sl.lp, sizeof(int32_t) * cols));
        HIP_TRY(x, x->alloc(&x->retire, sizeof(RetireEntry) * cols));
        HIP_TRY(x, x->alloc(&x->moves, sizeof(MoveEntry) * cols));
        HIP_TRY(x, x->alloc(&x->fresh, sizeof(int32_t) * cols));
        HIP_TRY(x, x->alloc(&x->adm_rows, sizeof(int32_t) * cols));
        HIP_TRY(x, x->alloc(&x->adm_ctl, sizeof(SlotCtl) * cols));
        x->cap_slots = cols;
    }
    if (lps > x->cap_lps) {
        x->drop_graph();
        x->release(x->ctl, sizeof(SlotCtl) * x->cap_lps);
        x->release(x->rlog, sizeof(int32_t) * RESTART_LOG * x->cap_lps);
        x->cap_lps = 0;
        HIP_TRY(x, x->alloc(&x->ctl, sizeof(SlotCtl) * lps));
        HIP_TRY(x, x->alloc(&x->rlog, sizeof(int32_t) * RESTART_LOG * lps));
        x->cap_lps = lps;
    }
    const size_t part_need = (size_t)(x->npx + x->npy + 2) * NTERM * ld;
    if (part_need > x->cap_part) {
        x->drop_graph();
        x->release(x->part, x->cap_part * sizeof(double));
        x->cap_part = 0;
        HIP_TRY(x, x->alloc(&x->part, part_need * sizeof(double)));
        x->cap_part = part_need;
    }
    *ld_out = ld;
    return PDLPB_OK;
}

// Device bytes of an allocation of `bytes` (the allocator rounds zero up).
int64_t alloc_bytes(size_t bytes) { return (int64_t)(bytes == 0 ? 256 : bytes); }

// Device bytes of the batch storage for `cols` columns (stride ld) and `rows`
// result rows: the eight iterate blocks, the per-slot arrays, the compaction
// plan and admission staging, the evaluation partial sums, the four result
// blocks and the per-LP control rows.  Mirrors resize_storage.
int64_t storage_bytes(const pdlpb_ctx* x, int32_t cols, int32_t rows) {
    const size_t esz = x->fp32 ? sizeof(float) : sizeof(double);
    const int32_t ld = ld_for(x, cols);
    int64_t b = 0;
    for (int q = 0; q < 8; ++q) b += alloc_bytes((size_t)(q < 4 ? x->n : x->m) * ld * esz);
    const size_t per_slot[] = {sizeof(SlotKey), sizeof(double), sizeof(double), sizeof(double),
                               sizeof(int32_t), sizeof(int32_t), sizeof(RetireEntry),
                               sizeof(MoveEntry), sizeof(int32_t), sizeof(int32_t),
                               sizeof(SlotCtl)};
    for (size_t e : per_slot) b += alloc_bytes(e * cols);
    b += alloc_bytes((size_t)(x->npx + x->npy + 2) * NTERM * ld * sizeof(double));
    for (int q = 0; q < 4; ++q) b += alloc_bytes((size_t)rows * (q < 2 ? x->n : x->m) * esz);
    b += alloc_bytes(sizeof(SlotCtl) * rows);
    b += alloc_bytes(sizeof(int32_t) * RESTART_LOG * rows);
    return b;
}

// Bytes currently held by the batch storage.
int64_t held_storage_bytes(const pdlpb_ctx* x) {
    int64_t b = 0;
    const void* ptrs[] = {x->blk[0], x->blk[1], x->blk[2], x->blk[3], x->blk[4], x->blk[5],
                          x->blk[6], x->blk[7], x->sl.key, x->sl.tau, x->sl.sigma, x->sl.dval,
                          x->sl.t_start, x->sl.lp, x->retire, x->moves, x->fresh, x->adm_rows,
                          x->adm_ctl, x->part, x->res[0], x->res[1], x->res[2], x->res[3],
                          x->ctl, x->rlog};
    for (const void* p : ptrs) {
        auto it = x->dev_sizes.find(const_cast<void*>(p));
        if (p && it != x->dev_sizes.end()) b += (int64_t)it->second;
    }
    return b;
}

// Serving storage: `cols` columns and `rows` result rows, keeping the first
// `keep_cols` columns of every block and slot array and the first
// min(rows, old rows) result and control rows.  New buffers are allocated and
// filled on the context's stream before the old ones go.
int resize_storage(pdlpb_ctx* x, int32_t cols, int32_t rows, int32_t keep_cols) {
    const int32_t n = x->n, m = x->m;
    const size_t esz = x->fp32 ? sizeof(float) : sizeof(double);
    const int32_t old_cols = x->cap_slots, old_ld = x->ld, old_rows = x->cap_lps;
    keep_cols = std::min(keep_cols, std::min(old_cols, cols));
    const int32_t keep_rows = std::min(old_rows, rows);
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    x->drop_graph();
    if (cols != old_cols || x->blk[0] == nullptr) {
        const int32_t ld = ld_for(x, cols);
        x->vec_ld = vec_for(x, cols);
        void* nb[8] = {};
        for (int q = 0; q < 8; ++q) {
            const int32_t r = q < 4 ? n : m;
            HIP_TRY(x, x->alloc(&nb[q], (size_t)r * ld * esz));
            if (keep_cols > 0 && r > 0 && x->blk[q])
                HIP_TRY(x, hipMemcpy2DAsync(nb[q], (size_t)ld * esz, x->blk[q], (size_t)old_ld * esz,
                                            (size_t)keep_cols * esz, (size_t)r,
                                            hipMemcpyDeviceToDevice, x->stream));
        }
        auto regrow = [&](auto*& p, size_t elem, bool copy) -> int {
            using E = std::remove_pointer_t<std::remove_reference_t<decltype(p)>>;
            E* q = nullptr;
            HIP_TRY(x, x->alloc(&q, elem * (size_t)cols));
            if (copy && keep_cols > 0 && p)
                HIP_TRY(x, hipMemcpyAsync(q, p, elem * (size_t)keep_cols, hipMemcpyDeviceToDevice,
                                          x->stream));
            HIP_TRY(x, hipStreamSynchronize(x->stream));
            x->release(p, 0);
            p = q;
            return PDLPB_OK;
        };
        int rc = PDLPB_OK;
        if (!rc) rc = regrow(x->sl.key, sizeof(SlotKey), true);
        if (!rc) rc = regrow(x->sl.tau, sizeof(double), true);
        if (!rc) rc = regrow(x->sl.sigma, sizeof(double), true);
        if (!rc) rc = regrow(x->sl.dval, sizeof(double), true);
        if (!rc) rc = regrow(x->sl.t_start, sizeof(int32_t), true);
        if (!rc) rc = regrow(x->sl.lp, sizeof(int32_t), true);
        if (!rc) rc = regrow(x->retire, sizeof(RetireEntry), false);
        if (!rc) rc = regrow(x->moves, sizeof(MoveEntry), false);
        if (!rc) rc = regrow(x->fresh, sizeof(int32_t), false);
        if (!rc) rc = regrow(x->adm_rows, sizeof(int32_t), false);
        if (!rc) rc = regrow(x->adm_ctl, sizeof(SlotCtl), false);
        if (rc) return rc;
        double* np_ = nullptr;
        const size_t part_need = (size_t)(x->npx + x->npy + 2) * NTERM * ld;
        HIP_TRY(x, x->alloc(&np_, part_need * sizeof(double)));
        HIP_TRY(x, hipStreamSynchronize(x->stream));
        for (int q = 0; q < 8; ++q) {
            void* old = x->blk[q];
            x->release(old, 0);
            x->blk[q] = nb[q];
        }
        x->release(x->part, 0);
        x->part = np_;
        x->cap_part = part_need;
        x->cap_slots = cols;
        x->cap_block_bytes = (size_t)ld * esz;
        x->ld = ld;
    }
    if (rows != old_rows || x->ctl == nullptr) {
        void* nr[4] = {};
        for (int q = 0; q < 4; ++q) {
            const size_t len = (size_t)(q < 2 ? n : m) * esz;
            HIP_TRY(x, x->alloc(&nr[q], len * rows));
            if (keep_rows > 0 && len > 0 && x->res[q])
                HIP_TRY(x, hipMemcpyAsync(nr[q], x->res[q], len * keep_rows,
                                          hipMemcpyDeviceToDevice, x->stream));
        }
        SlotCtl* nc = nullptr;
        int32_t* nl = nullptr;
        HIP_TRY(x, x->alloc(&nc, sizeof(SlotCtl) * rows));
        HIP_TRY(x, x->alloc(&nl, sizeof(int32_t) * RESTART_LOG * rows));
        if (keep_rows > 0 && x->ctl) {
            HIP_TRY(x, hipMemcpyAsync(nc, x->ctl, sizeof(SlotCtl) * keep_rows,
                                      hipMemcpyDeviceToDevice, x->stream));
            HIP_TRY(x, hipMemcpyAsync(nl, x->rlog, sizeof(int32_t) * RESTART_LOG * keep_rows,
                                      hipMemcpyDeviceToDevice, x->stream));
        }
        HIP_TRY(x, hipStreamSynchronize(x->stream));
        for (int q = 0; q < 4; ++q) {
            x->release(x->res[q], 0);
            x->res[q] = nr[q];
        }
        x->release(x->ctl, 0);
        x->release(x->rlog, 0);
        x->ctl = nc;
        x->rlog = nl;
        x->cap_res_x = (size_t)rows * n * esz;
        x->cap_res_y = (size_t)rows * m * esz;
        x->cap_lps = rows;
    }
    x->B = cols;
    return PDLPB_OK;
}

// Serving capacity targets: the next power of two at or above the need, within
// the session's limits (columns: max_batch; rows: result_capacity).
int32_t grow_target(int32_t have, int32_t need, int32_t limit) {
    if (need <= have) return have;
    return std::min(limit, std::max(need, next_pow2(need)));
}

// Columns and result rows the session needs once `extra` more LPs are
// submitted: every running and queued LP a column (up to max_batch), every row
// in use (rows are handed out from the free list in order) a result row.
void serve_need(const pdlpb_ctx* x, int32_t extra, int32_t* cols, int32_t* rows) {
    *cols = std::min<int64_t>(x->opt.max_batch, (int64_t)x->n_cols + (int64_t)x->queue.size() + extra);
    int32_t hi = x->row_hi;
    const int32_t nf = (int32_t)x->free_rows.size();
    for (int32_t k = 0; k < extra && k < nf; ++k) hi = std::max(hi, x->free_rows[nf - 1 - k] + 1);
    *rows = hi;
}

bool finite_all(const double* p, int64_t len) {
    for (int64_t i = 0; i < len; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

// ===========================================================================
extern "C" {

void pdlpb_default_options(pdlpb_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = (int32_t)sizeof(pdlpb_options);
    o->precision = PDLPB_FP64;
    o->restart_scope = PDLPB_RESTART_PER_LP;
    o->eval_every = 64;
    o->beta_sufficient = 0.2;
    o->beta_necessary = 0.8;
    o->beta_artificial = 0.36;
    o->theta = 0.5;
    o->step_size = 0.0;
    o->cross_sign = -1.0;
    o->infeas_tol = -1.0;
    o->dual_tol = -1.0;
    o->pw_ratio = 0;
    o->device = 0;
    o->stream = nullptr;
    o->max_batch = 4096;
    o->use_graphs = 1;
    o->tile_lanes = 0;
    o->tile_vec = 0;
    o->autotune = 1;
    o->tail_cols = 0;
}

int pdlpb_create(pdlpb_ctx** out, int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr,
                 const int32_t* col_idx, const double* val, const double* c, const double* b,
                 const char* sense, const double* l, const double* u, const pdlpb_options* opt) {
    auto bad = [](const std::string& s) {
        g_create_error = s;
        return PDLPB_EINVAL;
    };
    if (!out) return bad("out is NULL");
    *out = nullptr;
    pdlpb_options o;
    pdlpb_default_options(&o);
    if (opt) {
        if (opt->struct_size != (int32_t)sizeof(pdlpb_options))
            return bad("options.struct_size does not match this library");
        o = *opt;
    }
    if (m < 0 || n < 1) return bad("need m >= 0 and n >= 1");
    if (n >= VAR_NONE) return bad("n must be below 2^28 - 1");
    if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return bad("nnz must be in [0, 2^31)");
    if (!row_ptr || !c || !l || !u || (m > 0 && (!b || !sense)) ||
        (nnz > 0 && (!col_idx || !val)))
        return bad("NULL input array");
    if (o.precision != PDLPB_FP64 && o.precision != PDLPB_MIXED32) return bad("unknown precision");
    if (o.restart_scope != PDLPB_RESTART_PER_LP && o.restart_scope != PDLPB_RESTART_BATCH_AVG)
        return bad("unknown restart scope");
    if (o.eval_every < 2 || o.eval_every > 4096) return bad("eval_every must be in [2, 4096]");
    if (!(o.beta_sufficient >= 0 && o.beta_necessary >= 0 && o.beta_artificial >= 0 &&
          o.theta >= 0 && o.theta <= 1))
        return bad("restart parameters out of range");
    if (!(o.step_size >= 0.0) || !std::isfinite(o.step_size)) return bad("step_size must be >= 0");
    if (o.cross_sign != -1.0 && o.cross_sign != 1.0) return bad("cross_sign must be -1 or +1");
    if (std::isnan(o.infeas_tol) || !std::isfinite(o.infeas_tol)) return bad("infeas_tol must be finite");
    if (!std::isfinite(o.dual_tol)) return bad("dual_tol must be finite");
    if (o.max_blocks < 0) return bad("max_blocks must be >= 0");
    if (o.scaling != 0 && o.scaling != 1) return bad("scaling must be 0 or 1");
    if (o.max_batch < 1 || o.max_batch > MAX_BATCH) return bad("max_batch must be in [1, 4096]");
    if (o.restart_scope == PDLPB_RESTART_BATCH_AVG && o.max_batch > 1024) o.max_batch = 1024;
    if (o.tile_lanes != 0 && (o.tile_lanes < 1 || o.tile_lanes > 64 ||
                              (o.tile_lanes & (o.tile_lanes - 1))))
        return bad("tile_lanes must be 0 or a power of two in [1, 64]");
    if (o.tile_vec != 0 && o.tile_vec != 1 && o.tile_vec != 2 && o.tile_vec != 4)
        return bad("tile_vec must be 0, 1, 2 or 4");
    if (o.tail_cols < 0 || o.tail_cols > 64) return bad("tail_cols must be in [0, 64]");
    if (o.shared_start < -1 || o.shared_start > 1) return bad("shared_start must be -1, 0 or 1");
    if (o.stop_every != 0 && o.stop_every != o.eval_every &&
        (o.stop_every < 2 || o.eval_every % o.stop_every != 0))
        return bad("stop_every must be 0 or a divisor >= 2 of eval_every");
    if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr))
        return bad("dev_alloc and dev_free must both be set or both be NULL");
    // CSR structure
    if (row_ptr[0] != 0) return bad("row_ptr[0] must be 0");
    for (int32_t i = 0; i < m; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return bad("row_ptr must be nondecreasing");
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (k >= nnz) return bad("row_ptr exceeds nnz");
            if (col_idx[k] < 0 || col_idx[k] >= n) return bad("column index out of range");
            if (k > row_ptr[i] && col_idx[k] <= col_idx[k - 1])
                return bad("column indices must be strictly increasing within a row");
        }
    }
    if (row_ptr[m] != nnz) return bad("row_ptr[m] must equal nnz");
    if (!finite_all(val, nnz)) return bad("matrix values must be finite");
    if (!finite_all(c, n)) return bad("objective must be finite");
    if (m > 0 && !finite_all(b, m)) return bad("right-hand side must be finite");
    std::vector<double> rl(m), ru(m);
    for (int32_t i = 0; i < m; ++i) {
        switch (sense[i]) {
            case 'E': rl[i] = b[i]; ru[i] = b[i]; break;
            case 'L': rl[i] = -INFINITY; ru[i] = b[i]; break;
            case 'G': rl[i] = b[i]; ru[i] = INFINITY; break;
            case 'N': rl[i] = -INFINITY; ru[i] = INFINITY; break;
            default: return bad(std::string("unknown row sense '") + sense[i] + "'");
        }
    }
    for (int32_t j = 0; j < n; ++j) {
        if (std::isnan(l[j]) || std::isnan(u[j])) return bad("variable bounds must not be NaN");
        if (l[j] == INFINITY || u[j] == -INFINITY) return bad("infinite bound on the wrong side");
        if (l[j] > u[j]) return bad("variable lower bound above upper bound");
    }

    pdlpb_ctx* x = new (std::nothrow) pdlpb_ctx();
    if (!x) {
        g_create_error = "out of host memory";
        return PDLPB_ENOMEM;
    }
    x->opt = o;
    x->m = m;
    x->n = n;
    x->nnz = nnz;
    x->fp32 = o.precision == PDLPB_MIXED32;
    x->device = o.device;
    auto dev_fail = [&](hipError_t e, const char* what) {
        g_create_error = std::string(what) + ": " + hipGetErrorString(e);
        free_all(x);
        return PDLPB_EDEVICE;
    };
    hipError_t e = hipSetDevice(o.device);
    if (e != hipSuccess) return dev_fail(e, "hipSetDevice");
    e = scratch_setup(o.device);
    if (e != hipSuccess) return dev_fail(e, "hipGetSymbolAddress(scratch)");
    {
        int lds = 0;
        e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, o.device);
        if (e != hipSuccess) return dev_fail(e, "hipDeviceGetAttribute");
        x->lds_max = lds;
    }
    if (o.stream) {
        x->stream = static_cast<hipStream_t>(o.stream);
    } else {
        e = hipStreamCreateWithFlags(&x->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return dev_fail(e, "hipStreamCreate");
        x->own_stream = true;
    }
    e = hipHostMalloc((void**)&x->h_pinned, sizeof(int32_t) * 16, hipHostMallocDefault);
    if (e != hipSuccess) return dev_fail(e, "hipHostMalloc");

    // diagonal scaling: from here on A, c, the row bounds and the variable bounds
    // are the scaled LP's (the host copies of the caller's bounds stay as given)
    const double* l_in = l;
    const double* u_in = u;
    std::vector<double> s_val, s_c, s_l, s_u, s_b;
    if (o.scaling == 1) {
        compute_scaling(m, n, row_ptr, col_idx, val, 10, x->h_dr, x->h_dc);
        x->scaled = true;
        s_val.resize((size_t)nnz);
        for (int32_t i = 0; i < m; ++i)
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
                s_val[k] = (x->h_dr[i] * val[k]) * x->h_dc[col_idx[k]];
        s_c.resize(n);
        s_l.resize(n);
        s_u.resize(n);
        for (int32_t j = 0; j < n; ++j) {
            s_c[j] = x->h_dc[j] * c[j];
            s_l[j] = l[j] / x->h_dc[j];
            s_u[j] = u[j] / x->h_dc[j];
        }
        s_b.resize(m);
        for (int32_t i = 0; i < m; ++i) {
            rl[i] = x->h_dr[i] * rl[i];
            ru[i] = x->h_dr[i] * ru[i];
            s_b[i] = x->h_dr[i] * b[i];
        }
        val = s_val.data();
        c = s_c.data();
        l = s_l.data();
        u = s_u.data();
        b = s_b.data();
    } else {
        x->h_dr.assign(m, 1.0);
        x->h_dc.assign(n, 1.0);
    }

    // A' in CSR (= A in CSC): counting sort by column keeps row order inside each column
    std::vector<int32_t> h_arp(m + 1), h_trp(n + 1, 0), h_tci(nnz);
    std::vector<double> h_tv(nnz);
    for (int32_t i = 0; i <= m; ++i) h_arp[i] = (int32_t)row_ptr[i];
    for (int64_t k = 0; k < nnz; ++k) h_trp[col_idx[k] + 1] += 1;
    for (int32_t j = 0; j < n; ++j) h_trp[j + 1] += h_trp[j];
    {
        std::vector<int32_t> pos(h_trp.begin(), h_trp.end() - 1);
        for (int32_t i = 0; i < m; ++i)
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                const int32_t p = pos[col_idx[k]]++;
                h_tci[p] = i;
                h_tv[p] = val[k];
            }
    }
    // shared start: a change of variable v qualifies when its column and the
    // rows through it are small enough for the per-LP kernels
    x->h_sp_ok.assign(n, 0);
    for (int32_t v = 0; v < n; ++v) {
        if (h_trp[v + 1] - h_trp[v] > SP_MAX_COL) continue;
        int64_t touch = 1;
        for (int32_t k = h_trp[v]; k < h_trp[v + 1]; ++k)
            touch += h_arp[h_tci[k] + 1] - h_arp[h_tci[k]];
        x->h_sp_ok[v] = touch <= SP_MAX_TOUCH ? 1 : 0;
    }
    auto up = [&](auto** dst, const auto* src, size_t count) -> hipError_t {
        using E = std::remove_pointer_t<std::remove_reference_t<decltype(*dst)>>;
        hipError_t r = x->alloc(dst, count * sizeof(E));
        if (r != hipSuccess) return r;
        if (count == 0) return hipSuccess;
        return hipMemcpy(*dst, src, count * sizeof(E), hipMemcpyHostToDevice);
    };
    if ((e = up(&x->a_rp, h_arp.data(), h_arp.size())) != hipSuccess) return dev_fail(e, "upload A");
    if ((e = up(&x->a_ci, col_idx, (size_t)nnz)) != hipSuccess) return dev_fail(e, "upload A");
    if ((e = up(&x->a_v64, val, (size_t)nnz)) != hipSuccess) return dev_fail(e, "upload A");
    if ((e = up(&x->t_rp, h_trp.data(), h_trp.size())) != hipSuccess) return dev_fail(e, "upload A'");
    if ((e = up(&x->t_ci, h_tci.data(), h_tci.size())) != hipSuccess) return dev_fail(e, "upload A'");
    if ((e = up(&x->t_v64, h_tv.data(), h_tv.size())) != hipSuccess) return dev_fail(e, "upload A'");
    if (x->fp32) {
        std::vector<float> a32(val, val + nnz), t32(h_tv.begin(), h_tv.end());
        if ((e = up(&x->a_v32, a32.data(), a32.size())) != hipSuccess) return dev_fail(e, "upload A");
        if ((e = up(&x->t_v32, t32.data(), t32.size())) != hipSuccess) return dev_fail(e, "upload A'");
    }
    // ELL heads of A and A' (16 wide) for a matrix where more than a tenth of
    // the rows are longer than 8; others are walked in CSR alone
    {
        auto head = [&](const int32_t* rp, const int32_t* ci, const double* v, int32_t rows,
                        int32_t* ew_out, int32_t** d_ci, double** d_v64, float** d_v32,
                        int32_t width) {
            int32_t ew = width;
            if (ew == 0) {
                int64_t longer = 0;
                for (int32_t r = 0; r < rows; ++r) longer += (rp[r + 1] - rp[r]) > 8;
                ew = (longer * 10 > (int64_t)rows) ? 16 : 0;
            }
            if (ew_out) *ew_out = ew;
            if (ew == 0) return hipSuccess;
            std::vector<int32_t> hci((size_t)rows * ew, -1);
            std::vector<double> hv((size_t)rows * ew, 0.0);
            for (int32_t r = 0; r < rows; ++r)
                for (int32_t k = rp[r], u = 0; k < rp[r + 1] && u < ew; ++k, ++u) {
                    hci[(size_t)r * ew + u] = ci[k];
                    hv[(size_t)r * ew + u] = v[k];
                }
            hipError_t r1 = up(d_ci, hci.data(), hci.size());
            if (r1 != hipSuccess) return r1;
            r1 = up(d_v64, hv.data(), hv.size());
            if (r1 != hipSuccess || !x->fp32) return r1;
            std::vector<float> h32(hv.begin(), hv.end());
            return up(d_v32, h32.data(), h32.size());
        };
        std::vector<int32_t> h_aci(col_idx, col_idx + nnz);
        if ((e = head(h_arp.data(), h_aci.data(), val, m, &x->a_ew, &x->a_eci, &x->a_ev64,
                      &x->a_ev32, 0)) != hipSuccess)
            return dev_fail(e, "upload A");
        if ((e = head(h_trp.data(), h_tci.data(), h_tv.data(), n, &x->t_ew, &x->t_eci,
                      &x->t_ev64, &x->t_ev32, 0)) != hipSuccess)
            return dev_fail(e, "upload A'");
        // 8-wide copies for the persistent tail (small matrices only)
        if (nnz <= TAIL_MAX_NNZ && m > 0) {
            if ((e = head(h_arp.data(), h_aci.data(), val, m, nullptr, &x->a_e8ci, &x->a_e8v64,
                          &x->a_e8v32, 8)) != hipSuccess)
                return dev_fail(e, "upload A");
            if ((e = head(h_trp.data(), h_tci.data(), h_tv.data(), n, nullptr, &x->t_e8ci,
                          &x->t_e8v64, &x->t_e8v32, 8)) != hipSuccess)
                return dev_fail(e, "upload A'");
        }
    }
    if ((e = up(&x->c, c, (size_t)n)) != hipSuccess) return dev_fail(e, "upload c");
    if ((e = up(&x->xl, l, (size_t)n)) != hipSuccess) return dev_fail(e, "upload l");
    if ((e = up(&x->xu, u, (size_t)n)) != hipSuccess) return dev_fail(e, "upload u");
    if ((e = up(&x->rl, rl.data(), (size_t)m)) != hipSuccess) return dev_fail(e, "upload rows");
    if ((e = up(&x->ru, ru.data(), (size_t)m)) != hipSuccess) return dev_fail(e, "upload rows");
    {
        std::vector<int8_t> code(m);
        for (int32_t i = 0; i < m; ++i)
            code[i] = (int8_t)((std::isinf(rl[i]) && rl[i] < 0 ? 1 : 0) |
                               (std::isinf(ru[i]) && ru[i] > 0 ? 2 : 0));
        if ((e = up(&x->rcode, code.data(), (size_t)m)) != hipSuccess) return dev_fail(e, "upload rows");
    }
    if ((e = x->alloc(&x->g, sizeof(Globals))) != hipSuccess) return dev_fail(e, "alloc");

    x->h_xl.assign(l_in, l_in + n);
    x->h_xu.assign(u_in, u_in + n);
    if (x->scaled) {
        if ((e = up(&x->d_dr, x->h_dr.data(), (size_t)m)) != hipSuccess) return dev_fail(e, "upload");
        if ((e = up(&x->d_dc, x->h_dc.data(), (size_t)n)) != hipSuccess) return dev_fail(e, "upload");
    }
    double sc = 0.0, sb = 0.0;
    for (int32_t j = 0; j < n; ++j) sc += c[j] * c[j];
    for (int32_t i = 0; i < m; ++i) sb += b[i] * b[i];
    x->norm_c = std::sqrt(sc);
    x->norm_b = std::sqrt(sb);

    if (o.step_size > 0.0) {
        x->eta = o.step_size;
        x->norm_a = 0.0;
    } else {
        int rc = compute_opnorm(x, &x->norm_a);
        if (rc) {
            g_create_error = x->err;
            free_all(x);
            return rc;
        }
        x->eta = x->norm_a > 0.0 ? 0.998 / x->norm_a : 1.0;
    }
    Globals hg{};
    hg.eta = x->eta;
    hg.r_prev = -1.0;
    e = hipMemcpy(x->g, &hg, sizeof(Globals), hipMemcpyHostToDevice);
    if (e != hipSuccess) return dev_fail(e, "upload globals");
    x->pw_x = eval_rows_per_wave(n);
    x->pw_y = eval_rows_per_wave(m);
    x->npx = (n + 4 * x->pw_x - 1) / (4 * x->pw_x);
    x->npy = (m + 4 * x->pw_y - 1) / (4 * x->pw_y);
    *out = x;
    return PDLPB_OK;
}

int pdlpb_set_batch(pdlpb_ctx* x, int32_t B, const pdlpb_delta* deltas, const double* x_warm,
                    const double* y_warm, const double* w_warm, int32_t warm_mode, int32_t mem) {
    if (!x) return PDLPB_EINVAL;
    if (B < 1 || B > x->opt.max_batch) return x->fail(PDLPB_EINVAL, "B out of range [1, max_batch]");
    if (!deltas) return x->fail(PDLPB_EINVAL, "deltas is NULL");
    if (mem != PDLPB_MEM_HOST && mem != PDLPB_MEM_DEVICE) return x->fail(PDLPB_EINVAL, "unknown mem");
    if (warm_mode != PDLPB_WARM_NONE && warm_mode != PDLPB_WARM_SHARED &&
        warm_mode != PDLPB_WARM_PER_LP)
        return x->fail(PDLPB_EINVAL, "unknown warm mode");
    if (warm_mode != PDLPB_WARM_NONE && (!x_warm || (x->m > 0 && !y_warm)))
        return x->fail(PDLPB_EINVAL, "warm start vectors missing");
    if (x->ext_x && B > x->ext_cap)
        return x->fail(PDLPB_EINVAL, "batch larger than the result buffers (pdlpb_set_result_buffers)");
    HIP_TRY(x, hipSetDevice(x->device));
    if (x->launched) {
        // a serving block still in flight ends before its storage is reused
        HIP_TRY(x, hipStreamSynchronize(x->stream));
        x->launched = false;
    }
    const int32_t n = x->n, m = x->m;

    std::vector<pdlpb_delta> d(B);
    std::vector<double> w0(B, 0.0);
    if (mem == PDLPB_MEM_DEVICE) {
        HIP_TRY(x, hipMemcpy(d.data(), deltas, sizeof(pdlpb_delta) * B, hipMemcpyDeviceToHost));
        if (w_warm) HIP_TRY(x, hipMemcpy(w0.data(), w_warm, sizeof(double) * B, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(d.data(), deltas, sizeof(pdlpb_delta) * B);
        if (w_warm) std::memcpy(w0.data(), w_warm, sizeof(double) * B);
    }
    std::vector<SlotKey> h_key;
    std::vector<double> h_tau, h_sigma, h_dval;
    std::vector<int32_t> h_lp;
    std::vector<SlotCtl> hc(B);
    for (int32_t j = 0; j < B; ++j) {
        const pdlpb_delta& q = d[j];
        if (q.kind < PDLPB_BASE || q.kind > PDLPB_OBJ_UNIT)
            return x->fail(PDLPB_EINVAL, "delta kind out of range at LP " + std::to_string(j));
        if (q.kind != PDLPB_BASE && (q.var < 0 || q.var >= n))
            return x->fail(PDLPB_EINVAL, "delta var out of range at LP " + std::to_string(j));
        SlotKey key{};
        SlotCtl cl{};
        key.varkind = (q.kind == PDLPB_BASE ? VAR_NONE : q.var) | (q.kind << 28);
        int32_t status = lp_status(x, q);
        double w = default_weight(x, scaled_delta(x, q));
        if (w_warm) {
            w = w0[j];
            if (!(w > 0.0) || !std::isfinite(w)) status = PDLPB_STATUS_INVALID_INPUT;
        }
        if (status != PDLPB_STATUS_RUNNING) w = 1.0;
        key.flags = SLOT_ACTIVE;
        cl.w = w;
        cl.r_prev = -1.0;
        cl.status = status;
        for (double& v : cl.kkt) v = NAN;
        cl.obj = NAN;
        cl.dobj = NAN;
        if (status == PDLPB_STATUS_RUNNING) {   // running LPs fill slots [0, n_run0) in LP order
            h_key.push_back(key);
            h_tau.push_back(x->eta / w);
            h_sigma.push_back(x->eta * w);
            h_dval.push_back(scaled_delta(x, q).value);
            h_lp.push_back(j);
        } else {
            cl.iters = 0;
        }
        hc[j] = cl;
    }
    const int32_t n_run0 = (int32_t)h_key.size();

    // storage (grows, reused for smaller batches)
    int32_t ld = 0;
    {
        int rc = ensure_storage(x, B, B, &ld);
        if (rc) return rc;
    }
    {
        int rc = plan_shared_start(x, warm_mode, h_key, h_tau, h_sigma);
        if (rc) return rc;
    }
    const size_t esz = x->fp32 ? sizeof(float) : sizeof(double);
    // captured graphs stay valid: their keys hold the launch shapes, and
    // ensure_storage drops them when it moves a buffer
    // a batch ends any serving session: its queue, ids and results are dropped
    x->serving = false;
    x->queue.clear();
    x->completed.clear();
    x->id_row.clear();
    x->free_rows.clear();
    x->B = B;
    x->ld = ld;
    x->n_run0 = n_run0;
    x->h_delta = d;
    x->batch_set = true;
    x->solved = false;

    if (n_run0 > 0) {
        HIP_TRY(x, hipMemcpyAsync(x->sl.key, h_key.data(), sizeof(SlotKey) * n_run0,
                                  hipMemcpyHostToDevice, x->stream));
        HIP_TRY(x, hipMemcpyAsync(x->sl.tau, h_tau.data(), sizeof(double) * n_run0,
                                  hipMemcpyHostToDevice, x->stream));
        HIP_TRY(x, hipMemcpyAsync(x->sl.sigma, h_sigma.data(), sizeof(double) * n_run0,
                                  hipMemcpyHostToDevice, x->stream));
        HIP_TRY(x, hipMemcpyAsync(x->sl.dval, h_dval.data(), sizeof(double) * n_run0,
                                  hipMemcpyHostToDevice, x->stream));
        HIP_TRY(x, hipMemcpyAsync(x->sl.lp, h_lp.data(), sizeof(int32_t) * n_run0,
                                  hipMemcpyHostToDevice, x->stream));
    }
    HIP_TRY(x, hipMemcpyAsync(x->ctl, hc.data(), sizeof(SlotCtl) * B, hipMemcpyHostToDevice,
                              x->stream));
    // LPs that never run report x = 0, y = 0
    for (int32_t j = 0; j < B; ++j) {
        if (hc[j].status == PDLPB_STATUS_RUNNING) continue;
        for (int q = 0; q < 4; ++q) {
            const size_t len = (size_t)(q < 2 ? n : m) * esz;
            if (len)
                HIP_TRY(x, hipMemsetAsync(static_cast<char*>(x->out(q)) + (size_t)j * len, 0, len,
                                          x->stream));
        }
    }
    const double* xw = nullptr;
    const double* yw = nullptr;
    if (warm_mode != PDLPB_WARM_NONE) {
        const size_t nx = warm_mode == PDLPB_WARM_SHARED ? (size_t)n : (size_t)n * B;
        const size_t ny = warm_mode == PDLPB_WARM_SHARED ? (size_t)m : (size_t)m * B;
        if (mem == PDLPB_MEM_DEVICE && !x->scaled) {
            xw = x_warm;
            yw = y_warm;
        } else if (mem == PDLPB_MEM_DEVICE) {
            // the caller's vectors mapped to the scaled LP: x / dc, y / dr
            int rc = ensure_stage(x, nx + ny);
            if (rc) return rc;
            HIP_TRY(x, hipMemcpyAsync(x->stage, x_warm, nx * sizeof(double),
                                      hipMemcpyDeviceToDevice, x->stream));
            if (ny)
                HIP_TRY(x, hipMemcpyAsync(x->stage + nx, y_warm, ny * sizeof(double),
                                          hipMemcpyDeviceToDevice, x->stream));
            HIP_TRY(x, launch_rescale(x->stage, x->d_dc, (int64_t)nx, n, 1, x->stream));
            HIP_TRY(x, launch_rescale(x->stage + nx, x->d_dr, (int64_t)ny, m, 1, x->stream));
            xw = x->stage;
            yw = x->stage + nx;
        } else {
            int rc = ensure_stage(x, nx + ny);
            if (rc) return rc;
            HIP_TRY(x, hipMemcpyAsync(x->stage, x_warm, nx * sizeof(double), hipMemcpyHostToDevice,
                                      x->stream));
            if (ny)
                HIP_TRY(x, hipMemcpyAsync(x->stage + nx, y_warm, ny * sizeof(double),
                                          hipMemcpyHostToDevice, x->stream));
            if (x->scaled) {
                HIP_TRY(x, launch_rescale(x->stage, x->d_dc, (int64_t)nx, n, 1, x->stream));
                HIP_TRY(x, launch_rescale(x->stage + nx, x->d_dr, (int64_t)ny, m, 1, x->stream));
            }
            xw = x->stage;
            yw = x->stage + nx;
        }
    }
    if (x->sp_batch) {
        // the first iteration of the base LPs and of each change; the blocks are
        // written after the first evaluation, for the LPs that still run
        if (x->fp32) HIP_TRY(x, launch_sp_iterate<float>(shared_args<float>(x, xw, yw), x->stream));
        else HIP_TRY(x, launch_sp_iterate<double>(shared_args<double>(x, xw, yw), x->stream));
    } else if (x->fp32) {
        float* const* b = reinterpret_cast<float* const*>(x->blk);
        HIP_TRY(x, launch_init_blocks<float>(n, m, ld, n_run0, x->sl, x->xl, x->xu, xw,
                                             yw, warm_mode, b[0], b[1], b[4], b[5], x->stream));
    } else {
        double* const* b = reinterpret_cast<double* const*>(x->blk);
        HIP_TRY(x, launch_init_blocks<double>(n, m, ld, n_run0, x->sl, x->xl, x->xu,
                                              xw, yw, warm_mode, b[0], b[1], b[4], b[5],
                                              x->stream));
    }
    // host staging must outlive the copies
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    x->h_ctl = hc;
    return PDLPB_OK;
}

int pdlpb_solve(pdlpb_ctx* x, double tol, int64_t max_iters) {
    if (!x) return PDLPB_EINVAL;
    if (!x->batch_set) return x->fail(PDLPB_ESTATE, "no batch set");
    if (x->solved) return x->fail(PDLPB_ESTATE, "batch already solved; call pdlpb_set_batch");
    if (!(tol >= 0.0)) return x->fail(PDLPB_EINVAL, "tol must be >= 0");
    if (max_iters < 1 || max_iters > (1 << 30)) return x->fail(PDLPB_EINVAL, "max_iters out of range");
    HIP_TRY(x, hipSetDevice(x->device));
    int rc = PDLPB_OK;
    if (x->n_run0 > 0)
        rc = x->fp32 ? run_solve<float>(x, tol, (int32_t)max_iters)
                     : run_solve<double>(x, tol, (int32_t)max_iters);
    if (rc) return rc;
    rc = fetch_state(x);
    if (rc) return rc;
    x->solved = true;
    return PDLPB_OK;
}

int pdlpb_get(pdlpb_ctx* x, int32_t j, double* xo, double* yo, int32_t* status, double kkt[4],
              double* obj, int64_t* iters, int32_t mem) {
    if (!x) return PDLPB_EINVAL;
    if (!x->batch_set) return x->fail(PDLPB_ESTATE, "no batch set");
    if (j < 0 || j >= x->B) return x->fail(PDLPB_EINVAL, "LP index out of range");
    if (mem != PDLPB_MEM_HOST && mem != PDLPB_MEM_DEVICE) return x->fail(PDLPB_EINVAL, "unknown mem");
    if (!x->solved) return x->fail(PDLPB_ESTATE, "batch not solved yet");
    HIP_TRY(x, hipSetDevice(x->device));
    const SlotCtl& cl = x->h_ctl[j];
    if (status) *status = cl.status;
    if (kkt)
        for (int q = 0; q < 4; ++q) kkt[q] = cl.kkt[q];
    if (obj) *obj = cl.obj;
    if (iters) *iters = cl.iters;
    int rc = PDLPB_OK;
    if (xo) rc = copy_results(x, 0, j, 1, xo, mem);
    if (!rc && yo) rc = copy_results(x, 2, j, 1, yo, mem);
    return rc;
}

int pdlpb_set_result_buffers(pdlpb_ctx* x, double* X, double* Y, int32_t capacity) {
    if (!x) return PDLPB_EINVAL;
    if (!X && !Y) {
        x->ext_x = x->ext_y = nullptr;
        x->ext_cap = 0;
        x->batch_set = false;   // the last batch's results stay where they were written
        return PDLPB_OK;
    }
    if (!X || !Y) return x->fail(PDLPB_EINVAL, "set both result buffers or neither");
    if (x->fp32 || x->scaled)
        return x->fail(PDLPB_EINVAL, "result buffers need an FP64 context without scaling");
    if (capacity < 1 || capacity > x->opt.max_batch)
        return x->fail(PDLPB_EINVAL, "capacity out of range [1, max_batch]");
    x->ext_x = X;
    x->ext_y = Y;
    x->ext_cap = capacity;
    x->batch_set = false;       // results of an earlier batch are not in these buffers
    return PDLPB_OK;
}

int pdlpb_get_batch(pdlpb_ctx* x, double* X, double* Y, int32_t* status, double* kkt, double* obj,
                    int64_t* iters, int32_t mem) {
    if (!x) return PDLPB_EINVAL;
    if (!x->batch_set) return x->fail(PDLPB_ESTATE, "no batch set");
    if (!x->solved) return x->fail(PDLPB_ESTATE, "batch not solved yet");
    if (mem != PDLPB_MEM_HOST && mem != PDLPB_MEM_DEVICE) return x->fail(PDLPB_EINVAL, "unknown mem");
    HIP_TRY(x, hipSetDevice(x->device));
    const int32_t B = x->B;
    for (int32_t j = 0; j < B; ++j) {
        const SlotCtl& cl = x->h_ctl[j];
        if (status) status[j] = cl.status;
        if (kkt)
            for (int q = 0; q < 4; ++q) kkt[4 * (size_t)j + q] = cl.kkt[q];
        if (obj) obj[j] = cl.obj;
        if (iters) iters[j] = cl.iters;
    }
    int rc = PDLPB_OK;
    if (X) rc = copy_results(x, 0, 0, B, X, mem);
    if (!rc && Y) rc = copy_results(x, 2, 0, B, Y, mem);
    return rc;
}

}  // extern "C"

namespace {

// copy_results without an allocation: host destinations that need FP32
// widening or the scaling pass through the device's fixed staging array, as
// many LPs at a time as fit; every other case needs no staging.
int copy_results_noalloc(pdlpb_ctx* x, int q, int32_t count, double* dst, int32_t mem,
                         double* scr) {
    const int64_t rows = (q < 2) ? x->n : x->m;
    if (rows * count == 0) return PDLPB_OK;
    if (mem == PDLPB_MEM_DEVICE || (!x->fp32 && !x->scaled)) {
        // the library's own path, which stages nothing in these cases
        return copy_results(x, q, 0, count, dst, mem);
    }
    if ((size_t)rows > NOALLOC_DOUBLES)
        return x->fail(PDLPB_EINVAL, "one LP's vector (" + std::to_string(rows) +
                                         " doubles) exceeds the fixed staging array of " +
                                         std::to_string(NOALLOC_DOUBLES) + " doubles");
    const int32_t per = (int32_t)std::min<int64_t>(count, (int64_t)NOALLOC_DOUBLES / rows);
    const double* d = q < 2 ? x->d_dc : x->d_dr;
    for (int32_t c0 = 0; c0 < count; c0 += per) {
        const int32_t k = std::min(per, count - c0);
        const int64_t cnt = rows * k;
        if (x->fp32) {
            const float* src = static_cast<const float*>(x->out(q)) + (size_t)c0 * rows;
            HIP_TRY(x, launch_widen(src, cnt, scr, x->stream));
        } else {
            const double* src = static_cast<const double*>(x->out(q)) + (size_t)c0 * rows;
            HIP_TRY(x, hipMemcpyAsync(scr, src, cnt * sizeof(double), hipMemcpyDeviceToDevice,
                                      x->stream));
        }
        if (x->scaled) HIP_TRY(x, launch_rescale(scr, d, cnt, (int32_t)rows, 0, x->stream));
        HIP_TRY(x, hipMemcpyAsync(dst + (size_t)c0 * rows, scr, cnt * sizeof(double),
                                  hipMemcpyDeviceToHost, x->stream));
        // the next chunk reuses the array
        HIP_TRY(x, hipStreamSynchronize(x->stream));
    }
    return PDLPB_OK;
}

}  // namespace

extern "C" {

int pdlpb_get_batch_noalloc(pdlpb_ctx* x, double* X, double* Y, int32_t* status, double* kkt,
                            double* obj, int64_t* iters, int32_t mem) {
    if (!x) return PDLPB_EINVAL;
    if (!x->batch_set) return x->fail(PDLPB_ESTATE, "no batch set");
    if (!x->solved) return x->fail(PDLPB_ESTATE, "batch not solved yet");
    if (mem != PDLPB_MEM_HOST && mem != PDLPB_MEM_DEVICE) return x->fail(PDLPB_EINVAL, "unknown mem");
    if (x->device < 0 || x->device >= MAX_DEVICES) return x->fail(PDLPB_EINVAL, "device out of range");
    // one call at a time per process: the array is shared by every context on a device
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    double* scr = g_scratch_ptr[x->device];
    if (!scr) return x->fail(PDLPB_ESTATE, "staging array of the device not set up");
    HIP_TRY(x, hipSetDevice(x->device));
    const int32_t B = x->B;
    for (int32_t j = 0; j < B; ++j) {
        const SlotCtl& cl = x->h_ctl[j];
        if (status) status[j] = cl.status;
        if (kkt)
            for (int q = 0; q < 4; ++q) kkt[4 * (size_t)j + q] = cl.kkt[q];
        if (obj) obj[j] = cl.obj;
        if (iters) iters[j] = cl.iters;
    }
    int rc = PDLPB_OK;
    if (X) rc = copy_results_noalloc(x, 0, B, X, mem, scr);
    if (!rc && Y) rc = copy_results_noalloc(x, 2, B, Y, mem, scr);
    return rc;
}

int pdlpb_get_dual_objective(pdlpb_ctx* x, double* dual_obj) {
    if (!x) return PDLPB_EINVAL;
    if (!x->batch_set) return x->fail(PDLPB_ESTATE, "no batch set");
    if (!x->solved) return x->fail(PDLPB_ESTATE, "batch not solved yet");
    if (!dual_obj) return x->fail(PDLPB_EINVAL, "dual_obj is NULL");
    for (int32_t j = 0; j < x->B; ++j) dual_obj[j] = x->h_ctl[j].dobj;
    return PDLPB_OK;
}

int pdlpb_obbt_tighten(pdlpb_ctx* x, double eps, double min_improve, double* lo, double* hi,
                       int32_t* n_changed, int32_t* infeasible) {
    if (!x) return PDLPB_EINVAL;
    if (!x->batch_set) return x->fail(PDLPB_ESTATE, "no batch set");
    if (!x->solved) return x->fail(PDLPB_ESTATE, "batch not solved yet");
    if (!lo || !hi) return x->fail(PDLPB_EINVAL, "lo or hi is NULL");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return x->fail(PDLPB_EINVAL, "eps must be finite and >= 0");
    if (!(min_improve >= 0.0) || !std::isfinite(min_improve))
        return x->fail(PDLPB_EINVAL, "min_improve must be finite and >= 0");
    std::memcpy(lo, x->h_xl.data(), sizeof(double) * x->n);
    std::memcpy(hi, x->h_xu.data(), sizeof(double) * x->n);
    int32_t changed = 0, infeas = 0;
    for (int32_t j = 0; j < x->B; ++j) {
        const pdlpb_delta& q = x->h_delta[j];
        const SlotCtl& cl = x->h_ctl[j];
        if (q.kind != PDLPB_OBJ_UNIT || q.value == 0.0) continue;
        if (cl.status == PDLPB_STATUS_PRIMAL_INFEASIBLE) {   // the shared feasible set is empty
            infeas = 1;
            continue;
        }
        if (cl.status != PDLPB_STATUS_OPTIMAL || !std::isfinite(cl.dobj)) continue;
        // weak duality: value * x_var >= dobj; shift by Delta before dividing by value
        const double delta = eps * (1.0 + std::fabs(cl.obj) + std::fabs(cl.dobj));
        const double b = (cl.dobj - delta) / q.value;
        const int32_t v = q.var;
        if (q.value > 0.0 && b > lo[v] + min_improve) {
            lo[v] = b;
            ++changed;
        } else if (q.value < 0.0 && b < hi[v] - min_improve) {
            hi[v] = b;
            ++changed;
        }
    }
    if (n_changed) *n_changed = changed;
    if (infeasible) *infeasible = infeas;
    return PDLPB_OK;
}

int pdlpb_branch_scores(pdlpb_ctx* x, double parent_obj, double mu, double* gain, double* score) {
    if (!x) return PDLPB_EINVAL;
    if (!x->batch_set) return x->fail(PDLPB_ESTATE, "no batch set");
    if (!x->solved) return x->fail(PDLPB_ESTATE, "batch not solved yet");
    if (!std::isfinite(parent_obj)) return x->fail(PDLPB_EINVAL, "parent_obj must be finite");
    if (!(mu >= 0.0 && mu <= 1.0)) return x->fail(PDLPB_EINVAL, "mu must lie in [0, 1]");
    const int32_t B = x->B;
    std::vector<double> gn(B, NAN);
    std::unordered_map<int32_t, int32_t> first_up, first_down;
    for (int32_t j = 0; j < B; ++j) {
        const pdlpb_delta& q = x->h_delta[j];
        if (q.kind != PDLPB_SET_LO && q.kind != PDLPB_SET_HI) continue;
        const SlotCtl& cl = x->h_ctl[j];
        if (cl.status == PDLPB_STATUS_PRIMAL_INFEASIBLE || cl.status == PDLPB_STATUS_INFEASIBLE_BOUNDS)
            gn[j] = INFINITY;
        else if (cl.status == PDLPB_STATUS_OPTIMAL)
            gn[j] = std::max(cl.obj - parent_obj, 0.0);
        auto& first = q.kind == PDLPB_SET_LO ? first_up : first_down;
        first.emplace(q.var, j);
    }
    for (int32_t j = 0; j < B; ++j) {
        if (gain) gain[j] = gn[j];
        if (!score) continue;
        score[j] = NAN;
        const pdlpb_delta& q = x->h_delta[j];
        if (q.kind != PDLPB_SET_LO && q.kind != PDLPB_SET_HI) continue;
        const auto& other = q.kind == PDLPB_SET_LO ? first_down : first_up;
        auto it = other.find(q.var);
        if (it == other.end()) continue;
        const double a = gn[j], b = gn[it->second];
        if (std::isnan(a) || std::isnan(b)) continue;
        const double mn = std::min(a, b), mx = std::max(a, b);
        score[j] = std::isinf(mx) ? INFINITY : (1.0 - mu) * mn + mu * mx;
    }
    return PDLPB_OK;
}

int pdlpb_get_trace(pdlpb_ctx* x, int32_t j, double* x_iter, double* y_iter, double* w,
                    int32_t* restarts, int32_t* restart_log, int32_t log_cap) {
    if (!x) return PDLPB_EINVAL;
    if (!x->batch_set) return x->fail(PDLPB_ESTATE, "no batch set");
    if (!x->solved) return x->fail(PDLPB_ESTATE, "batch not solved yet");
    if (j < 0 || j >= x->B) return x->fail(PDLPB_EINVAL, "LP index out of range");
    HIP_TRY(x, hipSetDevice(x->device));
    const SlotCtl& cl = x->h_ctl[j];
    if (w) *w = cl.w;
    if (restarts) *restarts = cl.restarts;
    if (restart_log && log_cap > 0) {
        const int32_t cnt = std::min(std::min(cl.restarts, (int32_t)RESTART_LOG), log_cap);
        for (int32_t q = 0; q < cnt; ++q) restart_log[q] = x->h_rlog[(size_t)j * RESTART_LOG + q];
    }
    int rc = PDLPB_OK;
    if (x_iter) rc = copy_results(x, 1, j, 1, x_iter, PDLPB_MEM_HOST);
    if (!rc && y_iter) rc = copy_results(x, 3, j, 1, y_iter, PDLPB_MEM_HOST);
    return rc;
}


// ---------------------------------------------------------------------------
// serving: continuous batching
// ---------------------------------------------------------------------------

int pdlpb_set_base_warm(pdlpb_ctx* x, const double* xw, const double* yw, double w, int32_t mem) {
    if (!x) return PDLPB_EINVAL;
    if (!xw || (x->m > 0 && !yw)) return x->fail(PDLPB_EINVAL, "warm start vectors missing");
    if (!(w > 0.0) || !std::isfinite(w)) return x->fail(PDLPB_EINVAL, "w must be positive and finite");
    if (mem != PDLPB_MEM_HOST && mem != PDLPB_MEM_DEVICE) return x->fail(PDLPB_EINVAL, "unknown mem");
    HIP_TRY(x, hipSetDevice(x->device));
    if (!x->base_x) HIP_TRY(x, x->alloc(&x->base_x, sizeof(double) * ((size_t)x->n + x->m)));
    const hipMemcpyKind kind = mem == PDLPB_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                        : hipMemcpyHostToDevice;
    HIP_TRY(x, hipMemcpyAsync(x->base_x, xw, sizeof(double) * x->n, kind, x->stream));
    if (x->m)
        HIP_TRY(x, hipMemcpyAsync(x->base_x + x->n, yw, sizeof(double) * x->m, kind, x->stream));
    if (x->scaled) {
        HIP_TRY(x, launch_rescale(x->base_x, x->d_dc, x->n, x->n, 1, x->stream));
        HIP_TRY(x, launch_rescale(x->base_x + x->n, x->d_dr, x->m, x->m, 1, x->stream));
    }
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    x->base_w = w;
    x->have_base = true;
    return PDLPB_OK;
}

int pdlpb_serve_begin(pdlpb_ctx* x, int32_t result_capacity) {
    if (!x) return PDLPB_EINVAL;
    if (x->opt.restart_scope != PDLPB_RESTART_PER_LP)
        return x->fail(PDLPB_EINVAL, "serving needs the per-LP restart scope");
    if (result_capacity < 1 || result_capacity > (1 << 24))
        return x->fail(PDLPB_EINVAL, "result_capacity out of range");
    HIP_TRY(x, hipSetDevice(x->device));
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    // a session holds only what its LPs need: no narrow copies or shared-start
    // buffers of a batch
    x->drop_graph();
    free_narrow(x);
    free_shared_start(x);
    // storage starts at one column and one result row and grows with the LPs
    // submitted (pdlpb_serve_footprint, pdlpb_serve_trim)
    x->n_cols = 0;
    int rc = resize_storage(x, 1, 1, 0);
    if (rc) return rc;
    x->n_run0 = 0;
    x->batch_set = false;
    x->solved = false;
    if (!x->h_adm_pin) {
        const size_t bytes = 8 * sizeof(int32_t) + sizeof(RetireEntry) * (size_t)x->opt.max_batch;
        HIP_TRY(x, hipHostMalloc((void**)&x->h_adm_pin, bytes, hipHostMallocDefault));
    }
    x->adm_report = false;
    x->serving = true;
    x->res_cap = result_capacity;
    x->free_rows.clear();
    for (int32_t r = result_capacity - 1; r >= 0; --r) x->free_rows.push_back(r);
    x->row_id.assign(result_capacity, -1);
    x->row_state.assign(result_capacity, pdlpb_ctx::ROW_FREE);
    x->row_settled.assign(result_capacity, 0);
    x->settled_ctl.assign(result_capacity, SlotCtl{});
    x->row_hi = 0;
    x->id_row.clear();
    x->queue.clear();
    x->completed.clear();
    x->n_cols = 0;
    x->t0 = 0;
    x->launched = false;
    x->live = 1;
    choose_tile(x, 1);
    Globals hg{};
    hg.eta = x->eta;
    hg.r_prev = -1.0;
    HIP_TRY(x, hipMemcpy(x->g, &hg, sizeof(Globals), hipMemcpyHostToDevice));
    return PDLPB_OK;
}

int pdlpb_submit(pdlpb_ctx* x, int32_t count, const pdlpb_delta* deltas, int32_t warm_mode,
                 double tol, int64_t max_iters, int32_t mem, int64_t* first_id) {
    if (!x) return PDLPB_EINVAL;
    if (!x->serving) return x->fail(PDLPB_ESTATE, "call pdlpb_serve_begin first");
    if (count < 1 || !deltas) return x->fail(PDLPB_EINVAL, "need count >= 1 and deltas");
    if (warm_mode != PDLPB_WARM_NONE && warm_mode != PDLPB_WARM_BASE)
        return x->fail(PDLPB_EINVAL, "serving takes PDLPB_WARM_NONE or PDLPB_WARM_BASE");
    if (warm_mode == PDLPB_WARM_BASE && !x->have_base)
        return x->fail(PDLPB_ESTATE, "no base warm start set");
    if (!(tol >= 0.0)) return x->fail(PDLPB_EINVAL, "tol must be >= 0");
    if (max_iters < 1 || max_iters > (1 << 30)) return x->fail(PDLPB_EINVAL, "max_iters out of range");
    if (mem != PDLPB_MEM_HOST && mem != PDLPB_MEM_DEVICE) return x->fail(PDLPB_EINVAL, "unknown mem");
    if ((int64_t)x->free_rows.size() < count)
        return x->fail(PDLPB_ENOMEM, "not enough free result rows; release finished LPs");
    std::vector<pdlpb_delta> d(count);
    if (mem == PDLPB_MEM_DEVICE)
        HIP_TRY(x, hipMemcpy(d.data(), deltas, sizeof(pdlpb_delta) * count, hipMemcpyDeviceToHost));
    else
        std::memcpy(d.data(), deltas, sizeof(pdlpb_delta) * count);
    for (int32_t j = 0; j < count; ++j) {
        if (d[j].kind < PDLPB_BASE || d[j].kind > PDLPB_OBJ_UNIT)
            return x->fail(PDLPB_EINVAL, "delta kind out of range at LP " + std::to_string(j));
        if (d[j].kind != PDLPB_BASE && (d[j].var < 0 || d[j].var >= x->n))
            return x->fail(PDLPB_EINVAL, "delta var out of range at LP " + std::to_string(j));
    }
    *first_id = x->next_id;
    for (int32_t j = 0; j < count; ++j) {
        const pdlpb_delta& q = d[j];
        const int64_t id = x->next_id++;
        const int32_t row = x->free_rows.back();
        x->free_rows.pop_back();
        x->row_id[row] = id;
        x->id_row[id] = row;
        int32_t status = lp_status(x, q);
        // the base dual and weight belong to the base objective: objective changes
        // start from the base primal point only
        double w = (warm_mode == PDLPB_WARM_BASE && q.kind != PDLPB_OBJ_UNIT) ? x->base_w
                                                                               : default_weight(x, scaled_delta(x, q));
        x->row_hi = std::max(x->row_hi, row + 1);
        if (status != PDLPB_STATUS_RUNNING) {
            // settled without iterating: the outcome stays on the host (x = y = 0)
            SlotCtl cl{};
            cl.w = w;
            cl.status = status;
            for (double& v : cl.kkt) v = NAN;
            cl.obj = NAN;
            cl.dobj = NAN;
            cl.tol = tol;
            x->settled_ctl[row] = cl;
            x->row_settled[row] = 1;
            x->row_state[row] = pdlpb_ctx::ROW_STOPPED;
            x->completed.push_back(id);
            continue;
        }
        x->row_settled[row] = 0;
        x->row_state[row] = pdlpb_ctx::ROW_QUEUED;
        pdlpb_ctx::Pending p;
        p.row = row;
        p.varkind = (q.kind == PDLPB_BASE ? VAR_NONE : q.var) | (q.kind << 28);
        p.dval = scaled_delta(x, q).value;
        p.w = w;
        p.tol = tol;
        p.max_iters = (int32_t)max_iters;
        p.warm = warm_mode;
        x->queue.push_back(p);
    }
    return PDLPB_OK;
}

}  // extern "C"

namespace {

// admit queued LPs into free columns and run their first iteration (t_local = 0)
template <typename T>
int serve_admit(pdlpb_ctx* x) {
    const int32_t free_cols = x->B - x->n_cols;
    const int32_t k = std::min<int32_t>(free_cols, (int32_t)x->queue.size());
    if (k <= 0) return PDLPB_OK;
    // a batch admitted together shares one warm-start mode (the queue is split where it changes)
    const int32_t warm = x->queue.front().warm;
    int32_t cnt = 0;
    while (cnt < k && x->queue[cnt].warm == warm) ++cnt;
    const int32_t c0 = x->n_cols;
    x->h_adm_rows.resize(cnt);
    x->h_adm_ctl.resize(cnt);
    x->h_adm_key.resize(cnt);
    x->h_adm_tau.resize(cnt);
    x->h_adm_sigma.resize(cnt);
    x->h_adm_dval.resize(cnt);
    x->h_adm_tstart.resize(cnt);
    x->h_adm_lp.resize(cnt);
    for (int32_t j = 0; j < cnt; ++j) {
        const pdlpb_ctx::Pending p = x->queue.front();
        x->queue.pop_front();
        SlotKey key{};
        key.t_anchor = x->t0;
        key.t_end = x->t0 + p.max_iters - 1;
        key.varkind = p.varkind;
        key.flags = SLOT_ACTIVE | SLOT_NEW;
        x->h_adm_key[j] = key;
        x->h_adm_tau[j] = x->eta / p.w;
        x->h_adm_sigma[j] = x->eta * p.w;
        x->h_adm_dval[j] = p.dval;
        x->h_adm_tstart[j] = x->t0;
        x->h_adm_lp[j] = p.row;
        x->h_adm_rows[j] = p.row;
        x->row_state[p.row] = pdlpb_ctx::ROW_RUNNING;
        SlotCtl cl{};
        cl.w = p.w;
        cl.r_prev = -1.0;
        cl.status = PDLPB_STATUS_RUNNING;
        for (double& v : cl.kkt) v = NAN;
        cl.obj = NAN;
        cl.dobj = NAN;
        cl.tol = p.tol;
        x->h_adm_ctl[j] = cl;
    }
    const hipMemcpyKind h2d = hipMemcpyHostToDevice;
    HIP_TRY(x, hipMemcpyAsync(x->sl.key + c0, x->h_adm_key.data(), sizeof(SlotKey) * cnt, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.tau + c0, x->h_adm_tau.data(), sizeof(double) * cnt, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.sigma + c0, x->h_adm_sigma.data(), sizeof(double) * cnt, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.dval + c0, x->h_adm_dval.data(), sizeof(double) * cnt, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.t_start + c0, x->h_adm_tstart.data(), sizeof(int32_t) * cnt, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.lp + c0, x->h_adm_lp.data(), sizeof(int32_t) * cnt, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->adm_rows, x->h_adm_rows.data(), sizeof(int32_t) * cnt, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->adm_ctl, x->h_adm_ctl.data(), sizeof(SlotCtl) * cnt, h2d, x->stream));
    x->n_cols = c0 + cnt;
    HIP_TRY(x, launch_admit(x->ctl, x->adm_rows, x->adm_ctl, cnt, x->g, x->n_cols, x->stream));
    const double* xw = warm == PDLPB_WARM_BASE ? x->base_x : nullptr;
    const double* yw = warm == PDLPB_WARM_BASE ? x->base_x + x->n : nullptr;
    T* const* b = reinterpret_cast<T* const*>(x->blk);
    HIP_TRY(x, launch_init_columns<T>(x->n, x->m, x->ld, c0, cnt, x->sl, x->xl, x->xu, xw, yw,
                                      warm,
                                      b, x->stream));
    // first iteration of the admitted LPs at t = t0 (t_local = 0): a full evaluation
    const int32_t shape = shape_cols(x, x->n_cols);
    if (shape != x->live) {
        x->live = shape;
        choose_tile(x, shape);
    }
    int rc = enqueue_iteration<T>(x, 0, 2, nullptr, 1);
    if (!rc) rc = enqueue_evaluation<T>(x, 0, 1, 0, nullptr, 1);
    if (rc) return rc;
    // the admitted LPs that stopped at their first evaluation left in its
    // compaction; its plan goes to the host with the block, for serve_wait
    const hipMemcpyKind d2h = hipMemcpyDeviceToHost;
    HIP_TRY(x, hipMemcpyAsync(x->h_adm_pin, x->g, 8 * sizeof(int32_t), d2h, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->h_adm_pin + 8, x->retire, sizeof(RetireEntry) * x->n_cols, d2h,
                              x->stream));
    x->adm_report = true;
    return PDLPB_OK;
}

template <typename T>
int serve_launch(pdlpb_ctx* x) {
    // storage for every running and queued LP (no block is in flight here)
    int32_t need_cols = 0, need_rows = 0;
    serve_need(x, 0, &need_cols, &need_rows);
    const int32_t cols = grow_target(x->B, need_cols, x->opt.max_batch);
    const int32_t rows = grow_target(x->cap_lps, need_rows, x->res_cap);
    if (cols != x->B || rows != x->cap_lps) {
        const int rc0 = resize_storage(x, cols, rows, x->n_cols);
        if (rc0) return rc0;
    }
    int rc = serve_admit<T>(x);
    if (rc) return rc;
    if (x->n_cols == 0) return PDLPB_OK;
    const int32_t shape = shape_cols(x, x->n_cols);
    if (shape != x->live) {
        x->live = shape;
        choose_tile(x, shape);
    }
    if (x->opt.use_graphs && !x->timing) {
        rc = replay_epoch<T>(x);
        if (rc) return rc;
    } else {
        rc = enqueue_epoch<T>(x, nullptr);
        if (rc) return rc;
    }
    // the stopped LPs of this block, for the host's completion list
    HIP_TRY(x, hipMemcpyAsync(x->h_pinned, x->g, 8 * sizeof(int32_t), hipMemcpyDeviceToHost,
                              x->stream));
    if (!x->serve_ev) HIP_TRY(x, hipEventCreateWithFlags(&x->serve_ev, hipEventDisableTiming));
    HIP_TRY(x, hipEventRecord(x->serve_ev, x->stream));
    x->launched = true;
    return PDLPB_OK;
}

}  // namespace

extern "C" {

int pdlpb_serve_launch(pdlpb_ctx* x) {
    if (!x) return PDLPB_EINVAL;
    if (!x->serving) return x->fail(PDLPB_ESTATE, "call pdlpb_serve_begin first");
    if (x->launched) return x->fail(PDLPB_ESTATE, "previous block not waited for");
    HIP_TRY(x, hipSetDevice(x->device));
    return x->fp32 ? serve_launch<float>(x) : serve_launch<double>(x);
}

int pdlpb_serve_wait(pdlpb_ctx* x, int32_t* n_running, int32_t* n_queued) {
    if (!x) return PDLPB_EINVAL;
    if (!x->serving) return x->fail(PDLPB_ESTATE, "call pdlpb_serve_begin first");
    HIP_TRY(x, hipSetDevice(x->device));
    if (x->launched) {
        HIP_TRY(x, hipStreamSynchronize(x->stream));
        x->launched = false;
        x->t0 += x->opt.eval_every;
        if (x->adm_report) {
            // LPs that stopped at their first evaluation, as admitted in this block
            x->adm_report = false;
            const int32_t na = x->h_adm_pin[4];       // Globals::n_retire
            const RetireEntry* ae = reinterpret_cast<const RetireEntry*>(x->h_adm_pin + 8);
            for (int32_t k = 0; k < na; ++k) {
                x->row_state[ae[k].lp] = pdlpb_ctx::ROW_STOPPED;
                x->completed.push_back(x->row_id[ae[k].lp]);
            }
        }
        const int32_t nr = x->h_pinned[4];            // Globals::n_retire
        x->n_cols = x->h_pinned[3];                   // Globals::n_cols
        if (nr > 0) {
            x->h_retire.resize(nr);
            HIP_TRY(x, hipMemcpy(x->h_retire.data(), x->retire, sizeof(RetireEntry) * nr,
                                 hipMemcpyDeviceToHost));
            for (const RetireEntry& e : x->h_retire) {
                x->row_state[e.lp] = pdlpb_ctx::ROW_STOPPED;
                x->completed.push_back(x->row_id[e.lp]);
            }
        }
    }
    if (n_running) *n_running = x->n_cols;
    if (n_queued) *n_queued = (int32_t)x->queue.size();
    return PDLPB_OK;
}

int pdlpb_poll(pdlpb_ctx* x, int64_t* ids, int32_t cap, int32_t* count) {
    if (!x || !count) return PDLPB_EINVAL;
    int32_t c = 0;
    while (c < cap && !x->completed.empty()) {
        ids[c++] = x->completed.front();
        x->completed.pop_front();
    }
    *count = c;
    return PDLPB_OK;
}

int pdlpb_result(pdlpb_ctx* x, int64_t id, double* xo, double* yo, int32_t* status, double kkt[4],
                 double* obj, int64_t* iters, int32_t mem) {
    if (!x) return PDLPB_EINVAL;
    if (mem != PDLPB_MEM_HOST && mem != PDLPB_MEM_DEVICE) return x->fail(PDLPB_EINVAL, "unknown mem");
    auto it = x->id_row.find(id);
    if (it == x->id_row.end()) return x->fail(PDLPB_EINVAL, "unknown or released id");
    const int32_t row = it->second;
    if (x->row_state[row] != pdlpb_ctx::ROW_STOPPED) {
        // queued or running: the row may still hold another LP's data or be
        // written by the device, so nothing is read from it
        if (status) *status = PDLPB_STATUS_RUNNING;
        if (kkt)
            for (int q = 0; q < 4; ++q) kkt[q] = NAN;
        if (obj) *obj = NAN;
        if (iters) *iters = 0;
        return PDLPB_OK;
    }
    HIP_TRY(x, hipSetDevice(x->device));
    SlotCtl cl{};
    const bool settled = x->row_settled[row] != 0;
    if (settled) cl = x->settled_ctl[row];
    else HIP_TRY(x, hipMemcpy(&cl, x->ctl + row, sizeof(SlotCtl), hipMemcpyDeviceToHost));
    if (status) *status = cl.status;
    if (kkt)
        for (int q = 0; q < 4; ++q) kkt[q] = cl.kkt[q];
    if (obj) *obj = cl.obj;
    if (iters) *iters = cl.iters;
    if (settled) {
        // an LP that never iterated reports x = 0, y = 0
        for (int q = 0; q < 2; ++q) {
            double* d = q == 0 ? xo : yo;
            const size_t len = sizeof(double) * (size_t)(q == 0 ? x->n : x->m);
            if (!d || len == 0) continue;
            if (mem == PDLPB_MEM_DEVICE) HIP_TRY(x, hipMemsetAsync(d, 0, len, x->stream));
            else std::memset(d, 0, len);
        }
        HIP_TRY(x, hipStreamSynchronize(x->stream));
        return PDLPB_OK;
    }
    int rc = PDLPB_OK;
    if (xo) rc = copy_results(x, 0, row, 1, xo, mem);
    if (!rc && yo) rc = copy_results(x, 2, row, 1, yo, mem);
    return rc;
}

int pdlpb_release(pdlpb_ctx* x, int64_t id) {
    if (!x) return PDLPB_EINVAL;
    auto it = x->id_row.find(id);
    if (it == x->id_row.end()) return x->fail(PDLPB_EINVAL, "unknown or released id");
    const int32_t row = it->second;
    if (x->row_state[row] != pdlpb_ctx::ROW_STOPPED)
        return x->fail(PDLPB_ESTATE, "LP has not stopped; only a stopped LP's row can be released");
    x->id_row.erase(it);
    x->row_id[row] = -1;
    x->row_state[row] = pdlpb_ctx::ROW_FREE;
    x->row_settled[row] = 0;
    x->free_rows.push_back(row);
    while (x->row_hi > 0 && x->row_state[x->row_hi - 1] == pdlpb_ctx::ROW_FREE) --x->row_hi;
    return PDLPB_OK;
}

int pdlpb_serve_ready(pdlpb_ctx* x) {
    if (!x) return PDLPB_EINVAL;
    if (!x->serving) return x->fail(PDLPB_ESTATE, "call pdlpb_serve_begin first");
    if (!x->launched || !x->serve_ev) return 1;
    const hipError_t e = hipEventQuery(x->serve_ev);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return x->hip_fail(e, "hipEventQuery");
}

int pdlpb_serve_footprint(pdlpb_ctx* x, int32_t extra, int64_t* bytes) {
    if (!x || !bytes) return PDLPB_EINVAL;
    if (!x->serving) return x->fail(PDLPB_ESTATE, "call pdlpb_serve_begin first");
    if (extra < 0) return x->fail(PDLPB_EINVAL, "extra must be >= 0");
    int32_t need_cols = 0, need_rows = 0;
    serve_need(x, extra, &need_cols, &need_rows);
    const int32_t cols = grow_target(x->B, need_cols, x->opt.max_batch);
    const int32_t rows = grow_target(x->cap_lps, need_rows, x->res_cap);
    *bytes = x->dev_bytes - held_storage_bytes(x) + storage_bytes(x, cols, rows);
    return PDLPB_OK;
}

int pdlpb_serve_trim(pdlpb_ctx* x) {
    if (!x) return PDLPB_EINVAL;
    if (!x->serving) return x->fail(PDLPB_ESTATE, "call pdlpb_serve_begin first");
    if (x->launched) return x->fail(PDLPB_ESTATE, "a block is in flight; call pdlpb_serve_wait first");
    HIP_TRY(x, hipSetDevice(x->device));
    int32_t need_cols = 0, need_rows = 0;
    serve_need(x, 0, &need_cols, &need_rows);
    const int32_t cols = std::min(x->opt.max_batch, next_pow2(std::max(need_cols, 1)));
    const int32_t rows = std::min(x->res_cap, next_pow2(std::max(need_rows, 1)));
    if (cols >= x->B && rows >= x->cap_lps) return PDLPB_OK;
    return resize_storage(x, std::min(cols, x->B), std::min(rows, x->cap_lps), x->n_cols);
}

}  // extern "C"

namespace {

// Fused product launches at each width of `widths` on a batch of copies of the
// base LP; ms[i] receives the elapsed time of `reps` primal and `reps` dual
// launches after one untimed pair.
template <typename T>
int estimate_widths(pdlpb_ctx* x, const int32_t* widths, int32_t count, int32_t reps,
                    double* ms) {
    int32_t wmax = 1;
    for (int32_t i = 0; i < count; ++i) wmax = std::max(wmax, widths[i]);
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    int32_t ld = 0;
    int rc = ensure_storage(x, wmax, 1, &ld);
    if (rc) return rc;
    // the call replaces the batch: any batch or serving session ends
    x->serving = false;
    x->launched = false;
    x->queue.clear();
    x->completed.clear();
    x->id_row.clear();
    x->free_rows.clear();
    x->batch_set = false;
    x->solved = false;
    x->B = wmax;
    x->ld = ld;
    x->n_run0 = 0;
    std::vector<SlotKey> key(wmax);
    std::vector<double> step(wmax, x->eta), zero(wmax, 0.0);
    std::vector<int32_t> lp(wmax), t0(wmax, 0);
    for (int32_t s = 0; s < wmax; ++s) {
        key[s].t_anchor = 0;
        key[s].t_end = 1 << 30;
        key[s].varkind = VAR_NONE;
        key[s].flags = SLOT_ACTIVE;
        lp[s] = s;
    }
    const hipMemcpyKind h2d = hipMemcpyHostToDevice;
    HIP_TRY(x, hipMemcpyAsync(x->sl.key, key.data(), sizeof(SlotKey) * wmax, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.tau, step.data(), sizeof(double) * wmax, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.sigma, step.data(), sizeof(double) * wmax, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.dval, zero.data(), sizeof(double) * wmax, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.t_start, t0.data(), sizeof(int32_t) * wmax, h2d, x->stream));
    HIP_TRY(x, hipMemcpyAsync(x->sl.lp, lp.data(), sizeof(int32_t) * wmax, h2d, x->stream));
    Globals hg{};
    hg.n_cols = wmax;
    hg.n_active = wmax;
    hg.n_cols_next = wmax;
    hg.eta = x->eta;
    hg.r_prev = -1.0;
    HIP_TRY(x, hipMemcpyAsync(x->g, &hg, sizeof(Globals), h2d, x->stream));
    T* const* b = reinterpret_cast<T* const*>(x->blk);
    HIP_TRY(x, launch_init_blocks<T>(x->n, x->m, ld, wmax, x->sl, x->xl, x->xu, nullptr, nullptr,
                                     PDLPB_WARM_NONE, b[0], b[1], b[4], b[5], x->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(x, hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    hipError_t he = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return x->hip_fail(he, "hipEventCreate");
    }
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    for (int32_t i = 0; i < count; ++i) {
        x->live = widths[i];
        choose_tile(x, widths[i]);
        const StepArgs<T> p = step_args<T>(x, true, 1, 0);
        const StepArgs<T> d = step_args<T>(x, false, 1, 0);
        HIP_TRY(x, launch_primal<T>(p, x->tp.lanes, x->tp.vec, x->stream));
        HIP_TRY(x, launch_dual<T>(d, x->td.lanes, x->td.vec, x->stream));
        HIP_TRY(x, hipEventRecord(e0, x->stream));
        for (int32_t r = 0; r < reps; ++r) {
            HIP_TRY(x, launch_primal<T>(p, x->tp.lanes, x->tp.vec, x->stream));
            HIP_TRY(x, launch_dual<T>(d, x->td.lanes, x->td.vec, x->stream));
        }
        HIP_TRY(x, hipEventRecord(e1, x->stream));
        HIP_TRY(x, hipEventSynchronize(e1));
        float el = 0.f;
        HIP_TRY(x, hipEventElapsedTime(&el, e0, e1));
        ms[i] = (double)el;
    }
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    return PDLPB_OK;
}

}  // namespace

extern "C" {

int pdlpb_estimate_batch(pdlpb_ctx* x, const int32_t* widths, int32_t count, int32_t reps,
                         double* ms, int32_t* best) {
    if (!x) return PDLPB_EINVAL;
    if (!widths || count < 1) return x->fail(PDLPB_EINVAL, "need widths and count >= 1");
    if (reps < 1 || reps > 1000) return x->fail(PDLPB_EINVAL, "reps must be in [1, 1000]");
    for (int32_t i = 0; i < count; ++i)
        if (widths[i] < 1 || widths[i] > x->opt.max_batch)
            return x->fail(PDLPB_EINVAL, "width outside [1, max_batch]");
    HIP_TRY(x, hipSetDevice(x->device));
    std::vector<double> t(count, 0.0);
    const int rc = x->fp32 ? estimate_widths<float>(x, widths, count, reps, t.data())
                           : estimate_widths<double>(x, widths, count, reps, t.data());
    if (rc) return rc;
    // the width with the most column products per second (the paper's optimum)
    int32_t bi = 0;
    for (int32_t i = 1; i < count; ++i)
        if ((double)widths[i] / t[i] > (double)widths[bi] / t[bi]) bi = i;
    if (ms)
        for (int32_t i = 0; i < count; ++i) ms[i] = t[i];
    if (best) *best = widths[bi];
    return PDLPB_OK;
}

int pdlpb_set_tile(pdlpb_ctx* x, int32_t lanes, int32_t vec) {
    if (!x) return PDLPB_EINVAL;
    if (lanes != 0 && (lanes < 1 || lanes > 64 || (lanes & (lanes - 1))))
        return x->fail(PDLPB_EINVAL, "lanes must be 0 or a power of two in [1, 64]");
    if (vec != 0 && vec != 1 && vec != 2 && vec != 4)
        return x->fail(PDLPB_EINVAL, "vec must be 0, 1, 2 or 4");
    x->opt.tile_lanes = lanes;
    x->opt.tile_vec = vec;
    return PDLPB_OK;
}

int pdlpb_get_step_size(const pdlpb_ctx* x, double* eta, double* norm_a) {
    if (!x) return PDLPB_EINVAL;
    if (eta) *eta = x->eta;
    if (norm_a) *norm_a = x->norm_a;
    return PDLPB_OK;
}

int pdlpb_get_scaling(const pdlpb_ctx* x, double* dr, double* dc) {
    if (!x) return PDLPB_EINVAL;
    if (dr) std::copy(x->h_dr.begin(), x->h_dr.end(), dr);
    if (dc) std::copy(x->h_dc.begin(), x->h_dc.end(), dc);
    return PDLPB_OK;
}

int pdlpb_set_kernel_timing(pdlpb_ctx* x, int32_t enable) {
    if (!x) return PDLPB_EINVAL;
    x->timing = enable != 0;
    for (int q = 0; q < 5; ++q) {
        x->t_counts[q] = 0;
        x->t_ms[q] = 0.0;
        x->t_cols[q] = 0;
    }
    return PDLPB_OK;
}

int pdlpb_kernel_columns(pdlpb_ctx* x, int64_t cols[5]) {
    if (!x) return PDLPB_EINVAL;
    if (!cols) return x->fail(PDLPB_EINVAL, "cols is NULL");
    for (int q = 0; q < 5; ++q) cols[q] = x->t_cols[q];
    return PDLPB_OK;
}

int pdlpb_kernel_times(pdlpb_ctx* x, int64_t counts[5], double total_ms[5]) {
    if (!x) return PDLPB_EINVAL;
    for (int q = 0; q < 5; ++q) {
        if (counts) counts[q] = x->t_counts[q];
        if (total_ms) total_ms[q] = x->t_ms[q];
    }
    return PDLPB_OK;
}

int64_t pdlpb_device_bytes(const pdlpb_ctx* x) { return x ? x->dev_bytes : 0; }

int64_t pdlpb_graph_captures(const pdlpb_ctx* x) { return x ? x->graph_captures : 0; }

void pdlpb_destroy(pdlpb_ctx* x) { free_all(x); }

const char* pdlpb_last_error(const pdlpb_ctx* x) {
    return x ? x->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
