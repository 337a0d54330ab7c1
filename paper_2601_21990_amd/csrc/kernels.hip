// gfx950 kernels of the batched restarted PDHG solver.
//
// Dense blocks are row-major with row stride `ld`: element (row i, LP slot s)
// lives at i*ld + s, so one row of a block holds that row's entries of every
// LP of the batch contiguously.  A sparse row's product with a block is then
// a sum of contiguous row segments of the block, and a group of lanes that
// covers consecutive slots reads each segment with unit stride.
//
// Every lane sums its row's nonzeros sequentially in CSR order, whatever the
// tile shape, so each LP's arithmetic is independent of how many LPs share the
// batch and of the tile configuration.  All reductions are fixed-order trees
// (no atomics), so runs are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pdlpb.h"
#include "pdlpb_internal.h"

namespace pdlpb {

namespace {

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
    return fmax(fmin(v, hi), lo);
}
template <typename T>
__device__ __forceinline__ T clampt(T v, T lo, T hi) {
    return v > hi ? hi : (v < lo ? lo : v);   // max(min(v, hi), lo)
}

// Per-LP objective and variable bounds at variable i: the base vectors with
// the LP's single change applied (strong branching / bound tightening).
struct VarData {
    double c, lo, hi;
};
__device__ __forceinline__ VarData var_data(int32_t varkind, const double* dval, int32_t s,
                                            int32_t i, double c, double lo, double hi) {
    const int32_t kind = (int32_t)((uint32_t)varkind >> 28);
    VarData d{kind == PDLPB_OBJ_UNIT ? 0.0 : c, lo, hi};
    if (i == (varkind & VAR_MASK)) {
        const double v = dval[s];
        if (kind == PDLPB_SET_LO) d.lo = v;
        else if (kind == PDLPB_SET_HI) d.hi = v;
        else if (kind == PDLPB_OBJ_UNIT) d.c = v;
    }
    return d;
}

// Projection of one coordinate onto the barrier cone of [lo, hi] (Section 3):
// >= 0 if lo = -inf, <= 0 if hi = +inf, 0 if both, free otherwise.
__device__ __forceinline__ double barrier(double v, double lo, double hi) {
    if (isinf(lo) && lo < 0.0) v = fmax(v, 0.0);
    if (isinf(hi) && hi > 0.0) v = fmin(v, 0.0);
    return v;
}
// The same projection from the row's code (1: lo = -inf, 2: hi = +inf).
__device__ __forceinline__ double barrier_code(double v, int32_t code) {
    if (code & 1) v = fmax(v, 0.0);
    if (code & 2) v = fmin(v, 0.0);
    return v;
}
// Projection onto the recession cone of [lo, hi] (Section 4, infeasibility
// detection): free if both ends are infinite, >= 0 if only hi = +inf, <= 0 if
// only lo = -inf, 0 if both are finite.
__device__ __forceinline__ double recession(double v, double lo, double hi) {
    const bool li = isinf(lo) && lo < 0.0, hi_ = isinf(hi) && hi > 0.0;
    if (li && hi_) return v;
    if (hi_) return fmax(v, 0.0);
    if (li) return fmin(v, 0.0);
    return 0.0;
}
// One term of the support function phi_[lo,hi](v) = hi v_+ + lo v_- with 0 * inf = 0.
__device__ __forceinline__ double support1(double v, double lo, double hi) {
    return (v > 0.0 ? hi * v : 0.0) + (v < 0.0 ? lo * v : 0.0);
}

template <typename T, int VEC>
struct VecT;
template <typename T>
struct VecT<T, 1> {
    __device__ static void load(const T* p, T* out) { out[0] = p[0]; }
};
template <>
struct VecT<double, 2> {
    __device__ static void load(const double* p, double* out) {
        const double2 v = *reinterpret_cast<const double2*>(p);
        out[0] = v.x; out[1] = v.y;
    }
};
template <>
struct VecT<double, 4> {
    __device__ static void load(const double* p, double* out) {
        const double2 v = *reinterpret_cast<const double2*>(p);
        const double2 w = *reinterpret_cast<const double2*>(p + 2);
        out[0] = v.x; out[1] = v.y; out[2] = w.x; out[3] = w.y;
    }
};
template <>
struct VecT<float, 2> {
    __device__ static void load(const float* p, float* out) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        out[0] = v.x; out[1] = v.y;
    }
};
template <>
struct VecT<float, 4> {
    __device__ static void load(const float* p, float* out) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    }
};

// Row product of one sparse row with VEC consecutive columns of a block:
// acc[v] = sum_k a_k * G[col_k, s0 + v], nonzeros added in CSR order.  For a
// matrix with long rows (EW = 16) the first 16 nonzeros of every row sit in
// an ELL head (index -1 pads short rows), whose loads do not wait for the row
// pointers; gathers are issued CH at a time before the first one is used.
// Entries past the head (all entries when EW = 0) come from the CSR arrays,
// CH per trip.
constexpr int CH = 8;

template <typename T, int EW>
struct Head {
    int32_t j[EW];
    T a[EW];
};
template <typename T>
struct Head<T, 0> {};

template <typename T, int EW>
struct HeadVals;
template <int EW>
struct HeadVals<double, EW> {
    __device__ static void load(const double* p, double* out) {
        const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
        for (int i = 0; i < EW / 2; ++i) {
            const double2 w = q[i];
            out[2 * i] = w.x;
            out[2 * i + 1] = w.y;
        }
    }
};
template <int EW>
struct HeadVals<float, EW> {
    __device__ static void load(const float* p, float* out) {
        const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
        for (int i = 0; i < EW / 4; ++i) {
            const float4 w = q[i];
            out[4 * i] = w.x;
            out[4 * i + 1] = w.y;
            out[4 * i + 2] = w.z;
            out[4 * i + 3] = w.w;
        }
    }
};

// Everything one row of a step needs before its gathers: the row's CSR range
// and ELL head, the streamed block entries of the lane's slots and the row's
// base data.  None of it depends on the batch state, so a wave issues the
// loads of its first row together with those of the batch and slot state.
template <typename T, int VEC, int EW>
struct RowOps {
    int32_t kb, ke;
    T z[VEC], z0[VEC];
    double c, lo, hi;
    Head<T, EW> h;
};

template <typename T, int VEC, int EW, bool PRIMAL>
__device__ __forceinline__ void load_row(const StepArgs<T>& a, int32_t row, int32_t s0,
                                         RowOps<T, VEC, EW>& op) {
    op.kb = a.rp[row];
    op.ke = a.rp[row + 1];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        if (s0 + v < a.ncols) {
            const size_t e = (size_t)row * a.ld + s0 + v;
            op.z[v] = a.Z[e];
            op.z0[v] = a.Z0[e];
        }
    }
    op.c = PRIMAL ? a.c[row] : 0.0;
    op.lo = a.lo[row];
    op.hi = a.hi[row];
    if constexpr (EW > 0) {
        const int4* q = reinterpret_cast<const int4*>(a.eci + (size_t)row * EW);
#pragma unroll
        for (int i = 0; i < EW / 4; ++i) {
            const int4 w = q[i];
            op.h.j[4 * i] = w.x;
            op.h.j[4 * i + 1] = w.y;
            op.h.j[4 * i + 2] = w.z;
            op.h.j[4 * i + 3] = w.w;
        }
        HeadVals<T, EW>::load(a.ev + (size_t)row * EW, op.h.a);
    }
}

template <typename T, int VEC, int EW>
__device__ __forceinline__ void row_product(const StepArgs<T>& a, const RowOps<T, VEC, EW>& op,
                                            int32_t s0, T* acc) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = T(0);
    if constexpr (EW > 0) {
#pragma unroll
        for (int c0 = 0; c0 < EW; c0 += CH) {
            T g[CH][VEC];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                if (op.h.j[c0 + u] >= 0)
                    VecT<T, VEC>::load(a.G + (size_t)op.h.j[c0 + u] * a.ld + s0, g[u]);
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                if (op.h.j[c0 + u] >= 0) {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[v] = fma(op.h.a[c0 + u], g[u][v], acc[v]);
                }
            }
        }
    }
    const int32_t ke = op.ke;
    for (int32_t k0 = op.kb + EW; k0 < ke; k0 += CH) {
        int32_t j[CH];
        T w[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            j[u] = 0;
            w[u] = T(0);
            if (k0 + u < ke) {
                j[u] = a.ci[k0 + u];
                w[u] = a.av[k0 + u];
            }
        }
        T g[CH][VEC];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (k0 + u < ke) VecT<T, VEC>::load(a.G + (size_t)j[u] * a.ld + s0, g[u]);
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (k0 + u < ke) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] = fma(w[u], g[u][v], acc[v]);
            }
        }
    }
}

// The per-coordinate updates of one iteration, shared by every kernel that
// iterates, so that each computes the same bits.  No product is fused into a
// later addition.
// Primal (eq:main-iterate, first line; eq:mainiter): x^k rebuilt from the
// stored reflection z and the anchor x0, x~ = Pi_[lo,hi](x^k - tau (c + g)),
// reflection 2 x~ - x^k.
template <typename T>
__device__ __forceinline__ void primal_point(int32_t k, T z, T x0, T tau, double c, double lo,
                                             double hi, T g, T& xk, T& xt, T& xbar) {
#pragma clang fp contract(off)
    xk = (k == 0) ? x0 : T(double(k) / double(k + 1)) * z + x0 / T(k + 1);
    xt = clampt<T>(xk - tau * (T(c) + g), T(lo), T(hi));
    xbar = T(2) * xt - xk;
}
// Dual (eq:main-iterate, second line, Moreau form; eq:mainiter): q = y^k / sigma + v,
// y~ = sigma (q - Pi_[l,u](q)), y^{k+1} = wa (2 y~ - y^k) + y0 / wb.
template <typename T>
__device__ __forceinline__ void dual_point(T yk, T y0, T sg, T wa, T wb, T l, T u, T v, T& yt,
                                           T& ynext) {
#pragma clang fp contract(off)
    const T q = yk / sg + v;
    yt = sg * (q - clampt<T>(q, l, u));
    ynext = wa * (T(2) * yt - yk) + y0 / wb;
}
// Last Halpern iterate of a stopped LP, rebuilt from its reflection and anchor:
// a xbar + x0 / kp2 with a = (k+1)/(k+2), kp2 = k + 2 of its last iteration.
template <typename T>
__device__ __forceinline__ T halpern_last(double a, int32_t kp2, T xbar, T x0) {
#pragma clang fp contract(off)
    return T(a * (double)xbar + (double)x0 / (double)kp2);
}

// Halpern weights of eq:mainiter for inner index k: (k+1)/(k+2) and 1/(k+2).
__device__ __forceinline__ double halpern_a(int32_t k) { return double(k + 1) / double(k + 2); }

// Makes the kernel arguments that the first round of loads uses resident in
// scalar registers at entry, so they arrive in one batch instead of in the
// order the branches below would request them.
template <typename T>
__device__ __forceinline__ void fetch_args(const StepArgs<T>& a, const double* slot_step) {
    asm volatile("" ::"s"(a.rows), "s"(a.ncols), "s"(a.ld), "s"(a.wpb), "s"(a.it), "s"(a.g),
                 "s"(a.sl.key), "s"(slot_step), "s"(a.rp), "s"(a.Z), "s"(a.Z0), "s"(a.lo),
                 "s"(a.hi), "s"(a.eci), "s"(a.ev));
}

// Both step kernels start the same way.  A lane covers VEC slots from s0 of the
// rows RPW = 64/G apart that its wave visits; waves stride over row groups (the
// grid may hold fewer waves than groups).  The live column count, the lane's
// slot keys and step sizes, and the first row's operands are loaded in one
// round; only then do lanes past the live count, or whose slots all rest,
// leave.  Bounds on the host-side column count keep every load in the blocks.

// ---------------------------------------------------------------------------
// Primal step fused with G = A'Y (Section 5, eq:main-iterate, first line):
//   x^k  = x0                               if k == 0
//        = k/(k+1) Xbar + x0/(k+1)          otherwise (the Halpern average of
//                                           the previous iteration, eq:mainiter)
//   x~   = Pi_[xl_j, xu_j]( x^k - tau_j (c_j + (A'Y)_j) )
//   Xbar = 2 x~ - x^k                       (reflection, input of the dual step)
// Only Xbar is stored between iterations; x^{k+1} is rebuilt from Xbar and the
// anchor by the next launch, which saves one block write per iteration.
// ---------------------------------------------------------------------------
template <typename T, int G, int VEC, int EW>
__global__ __launch_bounds__(256) void k_primal(StepArgs<T> a) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    fetch_args(a, a.sl.tau);
    const int32_t s0 = blockIdx.y * (G * VEC) + (lane % G) * VEC;
    int32_t rw = (int32_t)blockIdx.x * a.wpb + wave;
    if (s0 >= a.ncols || rw * RPW >= a.rows) return;
    const int32_t wstride = (int32_t)gridDim.x * a.wpb;

    // one round of loads: batch state, slot state, first row (the batch state is
    // read through vector loads, which queue in order with the others)
    const __attribute__((address_space(1))) Globals* gv =
        (const __attribute__((address_space(1))) Globals*)a.g;
    asm volatile("" : "+v"(gv));
    const int32_t gcols = gv->n_cols;
    const int32_t t = gv->t0 + a.it;
    SlotKey key[VEC];
    double tau_d[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        if (s0 + v < a.ncols) {
            key[v] = a.sl.key[s0 + v];
            tau_d[v] = a.sl.tau[s0 + v];
        }
    }
    int32_t row = rw * RPW + lane / G;
    RowOps<T, VEC, EW> op;
    if (row < a.rows) load_row<T, VEC, EW, true>(a, row, s0, op);

    const int32_t ncols = min(a.ncols, gcols);
    if (s0 >= ncols) return;
    // per-slot operands: a lane keeps its slots for every row it visits
    bool live[VEC], last[VEC];
    int32_t varkind[VEC], kk[VEC];
    T tau[VEC];
    bool any = false;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        live[v] = false;
        last[v] = false;
        varkind[v] = VAR_NONE;
        kk[v] = 0;
        tau[v] = T(0);
        if (s0 + v < ncols) {
            live[v] = (key[v].flags & SLOT_ACTIVE) && t <= key[v].t_end &&
                      (!a.admit || (key[v].flags & SLOT_NEW));
            last[v] = (t == key[v].t_end);
            varkind[v] = key[v].varkind;
            kk[v] = t - key[v].t_anchor;
            tau[v] = T(tau_d[v]);
        }
        any = any || live[v];
    }
    if (!any) return;
    // z~ and the displacement are stored for the evaluation that reads them
    bool keep[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v)
        keep[v] = last[v] || a.eval == 2 || (a.eval == 1 && kk[v] == 0);

    auto step = [&](int32_t r, const RowOps<T, VEC, EW>& o) {
        T acc[VEC];
        row_product<T, VEC, EW>(a, o, s0, acc);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int32_t s = s0 + v;
            if (!live[v]) continue;
            const size_t e = (size_t)r * a.ld + s;
            const VarData d = var_data(varkind[v], a.sl.dval, s, r, o.c, o.lo, o.hi);
            const int32_t k = kk[v];
            T xk, xt, xbar;
            primal_point<T>(k, o.z[v], o.z0[v], tau[v], d.c, d.lo, d.hi, acc[v], xk, xt, xbar);
            a.Z[e] = xbar;
            if (keep[v]) {
                a.Zt[e] = xt;
                a.DZ[e] = xt - xk;
            }
        }
    };
    if (row < a.rows) step(row, op);
    for (rw += wstride; rw * RPW < a.rows; rw += wstride) {
        row = rw * RPW + lane / G;
        if (row >= a.rows) continue;
        RowOps<T, VEC, EW> o;
        load_row<T, VEC, EW, true>(a, row, s0, o);
        step(row, o);
    }
}

// ---------------------------------------------------------------------------
// Dual step fused with V = A Xbar (Section 5, eq:main-iterate, second line):
//   q   = y^k / sigma_j + V
//   y~  = sigma_j ( q - Pi_[l,u](q) )        (the printed expression in Moreau order)
//   y^{k+1} = (k+1)/(k+2) (2 y~ - y^k) + y0/(k+2)   (eq:mainiter)
// ---------------------------------------------------------------------------
template <typename T, int G, int VEC, int EW>
__global__ __launch_bounds__(256) void k_dual(StepArgs<T> a) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    fetch_args(a, a.sl.sigma);
    const int32_t s0 = blockIdx.y * (G * VEC) + (lane % G) * VEC;
    int32_t rw = (int32_t)blockIdx.x * a.wpb + wave;
    if (s0 >= a.ncols || rw * RPW >= a.rows) return;
    const int32_t wstride = (int32_t)gridDim.x * a.wpb;

    // one round of loads: batch state, slot state, first row (the batch state is
    // read through vector loads, which queue in order with the others)
    const __attribute__((address_space(1))) Globals* gv =
        (const __attribute__((address_space(1))) Globals*)a.g;
    asm volatile("" : "+v"(gv));
    const int32_t gcols = gv->n_cols;
    const int32_t t = gv->t0 + a.it;
    SlotKey key[VEC];
    double sig_d[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        if (s0 + v < a.ncols) {
            key[v] = a.sl.key[s0 + v];
            sig_d[v] = a.sl.sigma[s0 + v];
        }
    }
    int32_t row = rw * RPW + lane / G;
    RowOps<T, VEC, EW> op;
    if (row < a.rows) load_row<T, VEC, EW, false>(a, row, s0, op);

    const int32_t ncols = min(a.ncols, gcols);
    if (s0 >= ncols) return;
    bool live[VEC], keep[VEC];
    T sig[VEC], wa[VEC], wb[VEC];
    bool any = false;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        live[v] = false;
        keep[v] = false;
        sig[v] = T(1);
        wa[v] = T(0);
        wb[v] = T(1);
        if (s0 + v < ncols) {
            live[v] = (key[v].flags & SLOT_ACTIVE) && t <= key[v].t_end &&
                      (!a.admit || (key[v].flags & SLOT_NEW));
            const int32_t k = t - key[v].t_anchor;
            // y~ and the displacement are stored for the evaluation that reads them
            keep[v] = t == key[v].t_end || a.eval == 2 || (a.eval == 1 && k == 0);
            sig[v] = T(sig_d[v]);
            wa[v] = T(halpern_a(k));
            wb[v] = T(k + 2);
        }
        any = any || live[v];
    }
    if (!any) return;

    auto step = [&](int32_t r, const RowOps<T, VEC, EW>& o) {
        const T l = T(o.lo), u = T(o.hi);
        T acc[VEC];
        row_product<T, VEC, EW>(a, o, s0, acc);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            if (!live[v]) continue;
            const size_t e = (size_t)r * a.ld + s0 + v;
            const T yk = o.z[v];
            T yt, yn;
            dual_point<T>(yk, o.z0[v], sig[v], wa[v], wb[v], l, u, acc[v], yt, yn);
            a.Z[e] = yn;
            if (keep[v]) {
                a.Zt[e] = yt;
                a.DZ[e] = yt - yk;
            }
        }
    };
    if (row < a.rows) step(row, op);
    for (rw += wstride; rw * RPW < a.rows; rw += wstride) {
        row = rw * RPW + lane / G;
        if (row >= a.rows) continue;
        RowOps<T, VEC, EW> o;
        load_row<T, VEC, EW, false>(a, row, s0, o);
        step(row, o);
    }
}

// ---------------------------------------------------------------------------
// Evaluation: per-LP float64 sums for the fixed-point residual (eq:residual),
// the stopping measures (eq:stopping) and the primal-weight update.  A block
// of 4 waves owns a panel of 4*pw rows and 64 slots (one per lane); wave w
// sums rows [p0 + w*pw, p0 + (w+1)*pw) sequentially, then the four wave sums
// are added in wave order.  The panel size depends on the row count only, so
// each LP's sums do not depend on the batch around it.
// ---------------------------------------------------------------------------
// Operands of one evaluation row (x side: a column of A; y side: a row of A)
// for one LP slot, and the row's contribution to the evaluation sums.
struct XRow {
    double xt, dx, x0, c, lo, hi;
};
struct YRow {
    double yt, dy, y0, l, u;
};
// A row's operands as loaded, in the storage type of the blocks: a row fetched
// ahead is widened only when its terms are formed, so that its loads stay in
// flight behind the gathers of the current row.
template <typename T>
struct XRowIn {
    T xt, dx, x0;
    double c, lo, hi;
    __device__ XRow wide() const { return XRow{(double)xt, (double)dx, (double)x0, c, lo, hi}; }
};
template <typename T>
struct YRowIn {
    T yt, dy, y0;
    double l, u;
    __device__ YRow wide() const { return YRow{(double)yt, (double)dy, (double)y0, l, u}; }
};
// (KKT: a stopping test alone, which reads z~ only)
template <typename T, bool KKT = false>
__device__ __forceinline__ XRowIn<T> load_xrow(const EvalArgs<T>& a, int32_t i, int32_t s) {
    const size_t e = (size_t)i * a.ld + s;
    if constexpr (KKT) return XRowIn<T>{a.Xt[e], T(0), T(0), a.c[i], a.xl[i], a.xu[i]};
    return XRowIn<T>{a.Xt[e], a.DX[e], a.X0[e], a.c[i], a.xl[i], a.xu[i]};
}
template <typename T, bool KKT = false>
__device__ __forceinline__ YRowIn<T> load_yrow(const EvalArgs<T>& a, int32_t i, int32_t s) {
    const size_t e = (size_t)i * a.ld + s;
    if constexpr (KKT) return YRowIn<T>{a.Yt[e], T(0), T(0), a.rl[i], a.ru[i]};
    return YRowIn<T>{a.Yt[e], a.DY[e], a.Y0[e], a.rl[i], a.ru[i]};
}
// x side of column i: g = (A' y~)_i, h = (A' dy)_i, pdy = (A' Pi_B[l,u](dy))_i.
// tv receives the row's terms; callers add them to the running sums.  No
// product here is fused into a later addition, so every kernel that adds the
// same terms in the same order gets the same sums.
__device__ __forceinline__ void finish_xrow(const XRow& r, double g, double h, double pdy,
                                            int32_t varkind, const double* dval, int32_t s,
                                            int32_t i, double* tv) {
#pragma clang fp contract(off)
    const VarData d = var_data(varkind, dval, s, i, r.c, r.lo, r.hi);
    const double rc = barrier(-d.c - g, d.lo, d.hi);        // r~ (reduced cost at y~)
    const double rk = barrier(-d.c - (g - h), d.lo, d.hi);  // r at y^k = y~ - dy
    const double dr = barrier(rc - rk, d.lo, d.hi);
    const double dres = d.c + g + rc;
    const double ea = r.xt - r.x0;
    const double pr = pdy + dr;
    const double rx = r.dx - recession(r.dx, d.lo, d.hi);
    tv[0] = r.dx * r.dx;
    tv[1] = d.c * r.xt;
    tv[2] = support1(rc, d.lo, d.hi);
    tv[3] = dres * dres;
    tv[4] = d.c * d.c;
    tv[5] = ea * ea;
    tv[6] = support1(dr, d.lo, d.hi);
    tv[7] = pr * pr;
    tv[8] = d.c * r.dx;
    tv[9] = rx * rx;
}
// y side of row i: ax = (A x~)_i, adx = (A dx)_i; tv as above (terms 8, 9 zero)
__device__ __forceinline__ void finish_yrow(const YRow& r, double ax, double adx, double* tv) {
#pragma clang fp contract(off)
    const double pres = ax - clampd(ax, r.l, r.u);
    const double ea = r.yt - r.y0;
    const double ra = adx - recession(adx, r.l, r.u);
    tv[0] = r.dy * r.dy;
    tv[1] = r.dy * adx;
    tv[2] = support1(r.yt, r.l, r.u);
    tv[3] = pres * pres;
    tv[4] = ax * ax;
    tv[5] = ea * ea;
    tv[6] = support1(barrier(r.dy, r.l, r.u), r.l, r.u);
    tv[7] = ra * ra;
    tv[8] = 0.0;
    tv[9] = 0.0;
}
// The terms of a stopping test alone (eq:stopping: x side 1-4, y side 2-4),
// the same expressions as in finish_xrow / finish_yrow, from the products at
// z~ only; the other terms are 0 (the control pass reads none of them there).
__device__ __forceinline__ void finish_xrow_kkt(const XRow& r, double g, int32_t varkind,
                                                const double* dval, int32_t s, int32_t i,
                                                double* tv) {
#pragma clang fp contract(off)
    const VarData d = var_data(varkind, dval, s, i, r.c, r.lo, r.hi);
    const double rc = barrier(-d.c - g, d.lo, d.hi);        // r~ (reduced cost at y~)
    const double dres = d.c + g + rc;
#pragma unroll
    for (int q = 0; q < NTERM; ++q) tv[q] = 0.0;
    tv[1] = d.c * r.xt;
    tv[2] = support1(rc, d.lo, d.hi);
    tv[3] = dres * dres;
    tv[4] = d.c * d.c;
}
__device__ __forceinline__ void finish_yrow_kkt(const YRow& r, double ax, double* tv) {
#pragma clang fp contract(off)
    const double pres = ax - clampd(ax, r.l, r.u);
#pragma unroll
    for (int q = 0; q < NTERM; ++q) tv[q] = 0.0;
    tv[2] = support1(r.yt, r.l, r.u);
    tv[3] = pres * pres;
    tv[4] = ax * ax;
}

template <typename T, bool KKT>
__global__ __launch_bounds__(256) void k_eval(EvalArgs<T> a) {
    __shared__ double red[4][NTERM][64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int32_t s = blockIdx.y * 64 + lane;
    const bool xside = (int32_t)blockIdx.x < a.npx;
    const int32_t panel = xside ? blockIdx.x : blockIdx.x - a.npx;
    const int32_t pw = xside ? a.pw_x : a.pw_y;
    const int32_t rows = xside ? a.n : a.m;
    double acc[NTERM];
#pragma unroll
    for (int q = 0; q < NTERM; ++q) acc[q] = 0.0;

    // an evaluation of fresh cycles with none to evaluate (the last full one found none)
    if (!a.full && a.g->quiet) return;
    const int32_t ncols = min(a.ncols, a.g->n_cols);
    // between full evaluations only LPs at the start of a restart cycle (their
    // residual r(z^{n,0})) or at their last iteration read these sums
    bool need = false;
    if (s < ncols) {
        const SlotKey key = a.sl.key[s];
        const int32_t t = a.g->t0 + a.it;
        need = a.full || t == key.t_anchor || t >= key.t_end;
    }
    if (need) {
        const int32_t varkind = a.sl.key[s].varkind;
        const int32_t r0 = panel * 4 * pw + wave * pw;
        const int32_t r1 = min(r0 + pw, rows);
        // The wave walks the nonzeros of its rows as one stream, CH at a time,
        // so the gathers of short rows are in flight together; each row's
        // products still add its nonzeros in CSR order and the rows' terms
        // are added in row order, exactly as a row-by-row walk would.  Row
        // operands are loaded one row ahead.
        if (xside && r0 < r1) {
            const int32_t kbeg = a.t_rp[r0], kend = a.t_rp[r1];
            int32_t i = r0;
            int32_t ke = a.t_rp[r0 + 1];
            XRowIn<T> cur = load_xrow<T, KKT>(a, r0, s), nxt{};
            int32_t ke_n = 0;
            if (r0 + 1 < r1) {
                nxt = load_xrow<T, KKT>(a, r0 + 1, s);
                ke_n = a.t_rp[r0 + 2];
            }
            double g = 0.0, h = 0.0, pdy = 0.0;
            auto advance = [&]() {
                double tv[NTERM];
                if constexpr (KKT) finish_xrow_kkt(cur.wide(), g, varkind, a.sl.dval, s, i, tv);
                else finish_xrow(cur.wide(), g, h, pdy, varkind, a.sl.dval, s, i, tv);
#pragma unroll
                for (int q = 0; q < NTERM; ++q) acc[q] += tv[q];
                g = h = pdy = 0.0;
                ++i;
                cur = nxt;
                ke = ke_n;
                if (i + 1 < r1) {
                    nxt = load_xrow<T, KKT>(a, i + 1, s);
                    ke_n = a.t_rp[i + 2];
                }
            };
            for (int32_t k0 = kbeg; k0 < kend; k0 += CH) {
                // loads in the storage type; the widening to double waits
                // until every gather of the chunk has been issued
                int32_t jj[CH];
                T vv[CH], yv[CH], dv[CH];
                int32_t cd[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    jj[u] = 0;
                    vv[u] = T(0);
                    if (k0 + u < kend) {
                        jj[u] = a.t_ci[k0 + u];
                        vv[u] = a.t_v[k0 + u];
                    }
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    if (k0 + u < kend) {
                        const size_t f = (size_t)jj[u] * a.ld + s;
                        yv[u] = a.Yt[f];
                        if constexpr (!KKT) {
                            dv[u] = a.DY[f];
                            cd[u] = a.rcode[jj[u]];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    if (k0 + u < kend) {
                        while (k0 + u >= ke) advance();
                        const double w = (double)vv[u];
                        g = fma(w, (double)yv[u], g);
                        if constexpr (!KKT) {
                            const double d = (double)dv[u];
                            h = fma(w, d, h);
                            pdy = fma(w, barrier_code(d, cd[u]), pdy);
                        }
                    }
                }
            }
            while (i < r1) advance();
        } else if (r0 < r1) {
            const int32_t kbeg = a.a_rp[r0], kend = a.a_rp[r1];
            int32_t i = r0;
            int32_t ke = a.a_rp[r0 + 1];
            YRowIn<T> cur = load_yrow<T, KKT>(a, r0, s), nxt{};
            int32_t ke_n = 0;
            if (r0 + 1 < r1) {
                nxt = load_yrow<T, KKT>(a, r0 + 1, s);
                ke_n = a.a_rp[r0 + 2];
            }
            double ax = 0.0, adx = 0.0;                       // (A x~)_i, (A dx)_i
            auto advance = [&]() {
                double tv[NTERM];
                if constexpr (KKT) finish_yrow_kkt(cur.wide(), ax, tv);
                else finish_yrow(cur.wide(), ax, adx, tv);
#pragma unroll
                for (int q = 0; q < NTERM; ++q) acc[q] += tv[q];
                ax = adx = 0.0;
                ++i;
                cur = nxt;
                ke = ke_n;
                if (i + 1 < r1) {
                    nxt = load_yrow<T, KKT>(a, i + 1, s);
                    ke_n = a.a_rp[i + 2];
                }
            };
            for (int32_t k0 = kbeg; k0 < kend; k0 += CH) {
                int32_t jj[CH];
                T vv[CH], xv[CH], dv[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    jj[u] = 0;
                    vv[u] = T(0);
                    if (k0 + u < kend) {
                        jj[u] = a.a_ci[k0 + u];
                        vv[u] = a.a_v[k0 + u];
                    }
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    if (k0 + u < kend) {
                        const size_t f = (size_t)jj[u] * a.ld + s;
                        xv[u] = a.Xt[f];
                        if constexpr (!KKT) dv[u] = a.DX[f];
                    }
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    if (k0 + u < kend) {
                        while (k0 + u >= ke) advance();
                        const double w = (double)vv[u];
                        ax = fma(w, (double)xv[u], ax);
                        if constexpr (!KKT) adx = fma(w, (double)dv[u], adx);
                    }
                }
            }
            while (i < r1) advance();
        }
    }
#pragma unroll
    for (int q = 0; q < NTERM; ++q) red[wave][q][lane] = acc[q];
    __syncthreads();
    if (wave == 0 && s < ncols) {
        // layout [panel][term][slot]: a block writes its panel's sums as whole
        // rows of consecutive slots (one full cache line per 16 FP64 slots)
        double* out = (xside ? a.part_x : a.part_y) + (size_t)panel * NTERM * a.ld + s;
#pragma unroll
        for (int q = 0; q < NTERM; ++q) {
            const double v = ((red[0][q][lane] + red[1][q][lane]) + red[2][q][lane]) + red[3][q][lane];
            out[(size_t)q * a.ld] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Evaluation for narrow batches: the same sums as k_eval, bit for bit, with
// the lanes spread over rows instead of slots.  A block owns one panel and one
// slot (blockIdx.y); wave w owns the same rows [p0 + w*pw, p0 + (w+1)*pw) as in
// k_eval.  Its lanes take 64 consecutive rows at a time and compute each row's
// products (CSR order) and terms in parallel; lane q then adds term q of those
// rows in row order, continuing the wave's running sum, so every addition of
// k_eval happens in the same order.  The four wave sums are combined as there.
// ---------------------------------------------------------------------------
constexpr int NCH = 4;   // nonzeros of a row loaded together by k_eval_narrow

template <typename T, bool KKT>
__global__ __launch_bounds__(256) void k_eval_narrow(EvalArgs<T> a) {
    __shared__ double terms[4][64][NTERM + 1];
    __shared__ double red[4][NTERM];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // Workgroups go to the eight XCDs round robin (workgroup w to XCD w mod 8).
    // Numbering panel p's column c as 8 (ncols floor(p / 8) + c) + p mod 8 puts
    // every column of a panel on one XCD, one after another, so that they read
    // the panel's matrix rows and gathered lines from that XCD's L2.
    const int32_t w8 = (int32_t)(blockIdx.x & 7), q8 = (int32_t)(blockIdx.x >> 3);
    const int32_t s = q8 % a.ncols;
    const int32_t pidx = (q8 / a.ncols) * 8 + w8;
    if (pidx >= a.npx + a.npy) return;
    const bool xside = pidx < a.npx;
    const int32_t panel = xside ? pidx : pidx - a.npx;
    const int32_t pw = xside ? a.pw_x : a.pw_y;
    const int32_t rows = xside ? a.n : a.m;

    if (!a.full && a.g->quiet) return;
    const int32_t ncols = min(a.ncols, a.g->n_cols);
    if (s >= ncols) return;
    const SlotKey key = a.sl.key[s];
    const int32_t t = a.g->t0 + a.it;
    if (!(a.full || t == key.t_anchor || t >= key.t_end)) return;
    const int32_t varkind = key.varkind;
    const int32_t r0 = panel * 4 * pw + wave * pw;
    const int32_t r1 = min(r0 + pw, rows);
    double acc = 0.0;                      // lane q < NTERM: the wave's running sum of term q
    // every wave makes the same number of trips (pw is the same for all four),
    // so the block's barriers match even where a wave's rows run out
    for (int32_t off = 0; off < pw; off += 64) {
        const int32_t rb = r0 + off;
        const int32_t i = rb + lane;
        if (i < r1) {
            double tq[NTERM];
            if (xside) {
                const XRowIn<T> r = load_xrow<T, KKT>(a, i, s);
                double g = 0.0, h = 0.0, pdy = 0.0;
                const int32_t kb = a.t_rp[i], ke = a.t_rp[i + 1];
                // NCH nonzeros at a time: their indices, then their gathers, are
                // in flight together; the sums still add them in CSR order
                for (int32_t k0 = kb; k0 < ke; k0 += NCH) {
                    int32_t jj[NCH], cd[NCH];
                    T vv[NCH], yv[NCH], dv[NCH];
#pragma unroll
                    for (int u = 0; u < NCH; ++u) {
                        jj[u] = 0;
                        vv[u] = T(0);
                        if (k0 + u < ke) {
                            jj[u] = a.t_ci[k0 + u];
                            vv[u] = a.t_v[k0 + u];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < NCH; ++u) {
                        if (k0 + u < ke) {
                            const size_t f = (size_t)jj[u] * a.ld + s;
                            yv[u] = a.Yt[f];
                            if constexpr (!KKT) {
                                dv[u] = a.DY[f];
                                cd[u] = a.rcode[jj[u]];
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < NCH; ++u) {
                        if (k0 + u < ke) {
                            const double w = (double)vv[u];
                            g = fma(w, (double)yv[u], g);
                            if constexpr (!KKT) {
                                const double d = (double)dv[u];
                                h = fma(w, d, h);
                                pdy = fma(w, barrier_code(d, cd[u]), pdy);
                            }
                        }
                    }
                }
                if constexpr (KKT) finish_xrow_kkt(r.wide(), g, varkind, a.sl.dval, s, i, tq);
                else finish_xrow(r.wide(), g, h, pdy, varkind, a.sl.dval, s, i, tq);
            } else {
                const YRowIn<T> r = load_yrow<T, KKT>(a, i, s);
                double ax = 0.0, adx = 0.0;
                const int32_t kb = a.a_rp[i], ke = a.a_rp[i + 1];
                for (int32_t k0 = kb; k0 < ke; k0 += NCH) {
                    int32_t jj[NCH];
                    T vv[NCH], xv[NCH], dv[NCH];
#pragma unroll
                    for (int u = 0; u < NCH; ++u) {
                        jj[u] = 0;
                        vv[u] = T(0);
                        if (k0 + u < ke) {
                            jj[u] = a.a_ci[k0 + u];
                            vv[u] = a.a_v[k0 + u];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < NCH; ++u) {
                        if (k0 + u < ke) {
                            const size_t f = (size_t)jj[u] * a.ld + s;
                            xv[u] = a.Xt[f];
                            if constexpr (!KKT) dv[u] = a.DX[f];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < NCH; ++u) {
                        if (k0 + u < ke) {
                            const double w = (double)vv[u];
                            ax = fma(w, (double)xv[u], ax);
                            if constexpr (!KKT) adx = fma(w, (double)dv[u], adx);
                        }
                    }
                }
                if constexpr (KKT) finish_yrow_kkt(r.wide(), ax, tq);
                else finish_yrow(r.wide(), ax, adx, tq);
            }
#pragma unroll
            for (int q = 0; q < NTERM; ++q) terms[wave][lane][q] = tq[q];
        }
        __syncthreads();
        if (lane < NTERM) {
            const int32_t cnt = min(64, r1 - rb);
            for (int32_t j = 0; j < cnt; ++j) acc += terms[wave][j][lane];
        }
        __syncthreads();
    }
    if (lane < NTERM) red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && lane < NTERM) {
        double* out = (xside ? a.part_x : a.part_y) + (size_t)panel * NTERM * a.ld + s;
        const double v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        out[(size_t)lane * a.ld] = v;
    }
}

// sums[q][s] = sum over panels of part[panel][q][s]; q < NTERM: x side, else y side.
// One wave per (term, slot): lane l adds panels l, l+64, ... in order, then a
// butterfly over the 64 lanes (every lane ends with the same bits, since each
// level adds the same pair in either order).  The tree depends on the panel
// count only, not on the batch.
__global__ __launch_bounds__(256) void k_reduce(ControlArgs a) {
    const int32_t lane = threadIdx.x & 63;
    const int32_t pair = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pair >= 2 * NTERM * a.ncols) return;
    if (!a.full && !a.admit && !a.stop_only && a.g->quiet) return;
    const int32_t q = pair / a.ncols, s = pair % a.ncols;
    const bool xside = q < NTERM;
    const int32_t qq = xside ? q : q - NTERM;
    const int32_t np = xside ? a.npx : a.npy;
    const double* p = (xside ? a.part_x : a.part_y) + (size_t)qq * a.ld + s;
    const size_t stride = (size_t)NTERM * a.ld;
    double acc = 0.0;
    for (int32_t i = lane; i < np; i += 64) acc += p[(size_t)i * stride];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) a.sums[(size_t)q * a.ld + s] = acc;
}

// ---------------------------------------------------------------------------
// Control (Section 4: restarts, primal weight, stopping; Section 5: batched
// restart scope and per-LP stop).  One block; thread s handles slot s.
// ---------------------------------------------------------------------------
__device__ bool restart_due(double r, double r0, double r_prev, int32_t k, int32_t t,
                            const ControlArgs& a) {
#pragma clang fp contract(off)
    if (r <= a.beta_s * r0) return true;
    if (r_prev >= 0.0 && r <= a.beta_n * r0 && r > r_prev) return true;
    if ((double)k > a.beta_a * (double)t) return true;
    return false;
}

// eps-approximate infeasibility tests (Section 4, eq:primal-infeas, eq:dual-infeas)
// on the displacement sums of one LP: returns the status, or 0.
__device__ int32_t infeasible(const double* sx, const double* sy, int32_t ld, int32_t s,
                              double eps) {
#pragma clang fp contract(off)
    const double phi = sx[6 * ld + s] + sy[6 * ld + s];     // phi_[l,u](dy) + phi_box(dr)
    if (phi < 0.0 && sqrt(sx[7 * ld + s]) <= eps * fabs(phi)) return PDLPB_STATUS_PRIMAL_INFEASIBLE;
    const double cdx = sx[8 * ld + s];
    if (cdx < 0.0 && sqrt(sx[9 * ld + s]) <= eps * fabs(cdx) && sqrt(sy[7 * ld + s]) <= eps * fabs(cdx))
        return PDLPB_STATUS_DUAL_INFEASIBLE;
    return 0;
}

// new primal weight by exponential smoothing (Section 4), d from the anchor displacement
__device__ double smoothed_weight(double w, double dx2, double dy2, const ControlArgs& a) {
#pragma clang fp contract(off)
    const double dxn = sqrt(dx2), dyn = sqrt(dy2);
    const double num = a.pw_literal ? dxn : dyn;
    const double den = a.pw_literal ? dyn : dxn;
    if (num > 1e-10 && den > 1e-10 && isfinite(num) && isfinite(den))
        return exp(a.theta * log(num / den) + (1.0 - a.theta) * log(w));
    return w;
}

// restart bookkeeping of one LP: new weight and steps, cycle start, log
__device__ void restart_slot(const Slots& sl, int32_t s, SlotKey& key, SlotCtl& cl, int32_t* rlog,
                             int32_t t, double eta, double wn) {
    cl.w = wn;
    sl.tau[s] = eta / wn;
    sl.sigma[s] = eta * wn;
    key.t_anchor = t + 1;
    key.flags |= SLOT_FRESH;
    if (cl.restarts < RESTART_LOG) rlog[cl.restarts] = t - sl.t_start[s];
    cl.restarts += 1;
}

// Tests of one running LP at an evaluation (Section 4): the fixed-point
// residual, the stopping measures of eq:stopping, the infeasibility tests, the
// iteration limit and, with the per-LP restart scope, the restart rules and the
// primal-weight update.  sx / sy hold the LP's evaluation sums at
// [q * ld + s].  Returns 1 when the LP stopped (its status is recorded and its
// slot marked for retirement), else 0; *r_out and *resid_out give the residual
// and whether it was taken, for the batch-average scope.  No product is fused
// into a later addition, so every kernel calling this computes the same bits.
__device__ int32_t control_slot(const ControlArgs& a, bool full, bool stop, int32_t s,
                                SlotKey& st, SlotCtl& cl, int32_t* rlog, const double* sx,
                                const double* sy, int32_t ld, int32_t t, double eta, bool per_lp,
                                double* r_out, bool* resid_out) {
#pragma clang fp contract(off)
    // sx, sy point at the slot's sums: term q at [q * ld]
    const double tol = cl.tol;
    const int32_t k = t - st.t_anchor;
    const bool final_now = (t >= st.t_end);
    const double dx2 = sx[0 * ld], cx = sx[1 * ld], phix = sx[2 * ld];
    const double dres2 = sx[3 * ld], c2 = sx[4 * ld];
    const double dy2 = sy[0 * ld], cross = sy[1 * ld], phiy = sy[2 * ld];
    const double pres2 = sy[3 * ld], ax2 = sy[4 * ld];
    const double w = cl.w;
    // fixed-point residual r(z) = ||T(z) - z||_M (eq:residual, cross-term sign per option)
    const double q2 = (w / eta) * dx2 + (1.0 / (eta * w)) * dy2 + 2.0 * a.cross_sign * cross;
    const double r = isfinite(q2) ? sqrt(fmax(q2, 0.0)) : NAN;
    // stopping measures (eq:stopping)
    const double phis = phix + phiy;
    const double gap = isfinite(phis) ? fabs(cx + phis) / (1.0 + fabs(cx) + fabs(phis)) : INFINITY;
    const double pri = sqrt(pres2) / (1.0 + sqrt(ax2));
    const double dua = sqrt(dres2) / (1.0 + sqrt(c2));
    double rel = fmax(gap, fmax(pri, dua));
    if (isnan(gap) || isnan(pri) || isnan(dua)) rel = NAN;
    // an LP that ran out of budget before this evaluation is evaluated at its final z~
    const bool at_eval = (t <= st.t_end);
    const bool full_here = full && at_eval;
    // the stopping test runs at full evaluations and at the stopping tests in between
    const bool test_here = (full || stop) && at_eval;
    const bool resid_here = at_eval && (full || k == 0);
    // order of the tests: NaN, stopping, infeasibility, iteration limit
    const double eps_inf = a.infeas_tol < 0.0 ? tol : a.infeas_tol;
    const int32_t infeas = (full_here && eps_inf > 0.0) ? infeasible(sx, sy, ld, 0, eps_inf) : 0;
    int32_t status = PDLPB_STATUS_RUNNING;
    if ((resid_here && !isfinite(r)) || (test_here && !isfinite(rel))) {
        status = PDLPB_STATUS_NUMERICAL_ERROR;
    } else if (test_here && gap <= tol && pri <= tol && dua <= (a.dual_tol < 0.0 ? tol : a.dual_tol)) {
        status = PDLPB_STATUS_OPTIMAL;
    } else if (infeas) {
        status = infeas;
    } else if (final_now) {
        status = PDLPB_STATUS_ITERATION_LIMIT;
    }
    if (full || stop || k == 0 || final_now) {   // the evaluation computed this LP's sums
        cl.kkt[0] = gap; cl.kkt[1] = pri; cl.kkt[2] = dua; cl.kkt[3] = rel;
        cl.obj = cx;
        cl.dobj = -phis;
    }
    *r_out = r;
    *resid_out = resid_here;
    if (status != PDLPB_STATUS_RUNNING) {
        const int32_t t_last = t < st.t_end ? t : st.t_end;
        cl.status = status;
        cl.t_last = t_last;
        cl.k_last = t_last - st.t_anchor;
        cl.iters = t_last - a.sl.t_start[s] + 1;
        st.flags = SLOT_RETIRE;
        return 1;
    }
    if (!per_lp) return 0;
    if (k == 0) {
        if (resid_here) {
            cl.r0 = r;
            cl.r_prev = r;
        }
        st.flags &= ~SLOT_FRESH;
    } else if (full) {
        if (restart_due(r, cl.r0, cl.r_prev, k, t - a.sl.t_start[s], a)) {
            restart_slot(a.sl, s, st, cl, rlog, t, eta,
                         smoothed_weight(w, sx[5 * ld], sy[5 * ld], a));
            cl.r_prev = -1.0;
        } else {
            cl.r_prev = r;
        }
    }
    return 0;
}

// ---------------------------------------------------------------------------
// Control (Section 4: restarts, primal weight, stopping, infeasibility;
// Section 5: batched restart scope, per-LP stop and compaction).  One block;
// thread s handles slot s.  On full evaluations it also plans the compaction:
// stopped LPs are retired and running LPs beyond the new column count move
// into the freed slots, so the live columns stay a prefix [0, n_cols).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_control(ControlArgs a) {
    __shared__ double sh_r[1024];
    __shared__ int32_t sh_n[1024];
    __shared__ int32_t sh_flags[MAX_BATCH];
    __shared__ int32_t sh_flag;
    Globals* g = a.g;
    if (!a.full && !a.admit && !a.stop_only && g->quiet) return;
    const int32_t t = g->t0 + a.it;
    const int32_t nc = min(a.ncols, g->n_cols);
    const double eta = g->eta;
    const double* sx = a.sums;
    const double* sy = a.sums + (size_t)NTERM * a.ld;
    int32_t my_active = 0;
    if (a.batch_avg) {
        sh_r[threadIdx.x] = 0.0;
        sh_n[threadIdx.x] = 0;
    }
    __syncthreads();

    int32_t my_fresh = 0;   // running LPs that the next evaluation of fresh cycles reads
    // pass 1: stopping tests, residuals, per-LP restarts
    for (int32_t s = threadIdx.x; s < nc; s += blockDim.x) {
        SlotKey& st = a.sl.key[s];
        const int32_t lp = a.sl.lp[s];
        SlotCtl& cl = a.ctl[lp];
        if (!(st.flags & SLOT_ACTIVE)) continue;
        if (a.admit) {
            if (!(st.flags & SLOT_NEW)) {     // already running: not evaluated in this pass
                my_active += 1;
                continue;
            }
            st.flags &= ~SLOT_NEW;
        }
        double r = 0.0;
        bool resid_here = false;
        if (control_slot(a, a.full != 0, a.stop_only != 0, s, st, cl,
                         a.rlog + (size_t)lp * RESTART_LOG, sx + s, sy + s, a.ld, t, eta,
                         !a.batch_avg, &r, &resid_here))
            continue;
        my_active += 1;
        if (a.batch_avg && resid_here) {   // indexed by LP: the average adds LPs in LP order
            sh_r[lp] = r;
            sh_n[lp] = 1;
        }
        if ((st.flags & SLOT_FRESH) || st.t_end <= t + 1) my_fresh += 1;
    }

    // batch-average scope: mean residual over running LPs, shared decision
    if (a.batch_avg) {
        __syncthreads();
        if (threadIdx.x == 0) {
            double sum = 0.0;
            int32_t cnt = 0;
            for (int32_t i = 0; i < (int32_t)blockDim.x; ++i) {
                if (sh_n[i]) { sum += sh_r[i]; cnt += 1; }
            }
            const int32_t k = t - g->batch_k0;
            int32_t flag = 0;   // 0 nothing, 1 start of a cycle, 2 restart
            if (cnt > 0) {
                const double rbar = sum / (double)cnt;
                if (k == 0) {
                    g->r0 = rbar;
                    g->r_prev = rbar;
                    flag = 1;
                } else if (a.full) {
                    // LPs of one batch start together, so K = t
                    if (restart_due(rbar, g->r0, g->r_prev, k, t, a)) {
                        flag = 2;
                        g->batch_k0 = t + 1;
                        g->r_prev = -1.0;
                    } else {
                        g->r_prev = rbar;
                    }
                }
            }
            sh_flag = flag;
        }
        __syncthreads();
        const int32_t flag = sh_flag;
        for (int32_t s = threadIdx.x; s < nc; s += blockDim.x) {
            SlotKey& st = a.sl.key[s];
            if (!(st.flags & SLOT_ACTIVE)) continue;
            const int32_t lp = a.sl.lp[s];
            if (flag == 1 || (t - st.t_anchor) == 0) st.flags &= ~SLOT_FRESH;
            if (flag == 2) {
                SlotCtl& cl = a.ctl[lp];
                restart_slot(a.sl, s, st, cl, a.rlog + (size_t)lp * RESTART_LOG, t, eta,
                             smoothed_weight(cl.w, sx[5 * a.ld + s], sy[5 * a.ld + s], a));
            }
        }
    }

    // running count (fixed-order block sum)
    __syncthreads();
    sh_n[threadIdx.x] = my_active;
    __syncthreads();
    for (int32_t w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int32_t)threadIdx.x < w) sh_n[threadIdx.x] += sh_n[threadIdx.x + w];
        __syncthreads();
    }
    const int32_t n_run = sh_n[0];
    // a full pass decides whether the next evaluation of fresh cycles has work
    // (never skipped under the batch-average scope or after admissions)
    __syncthreads();
    sh_n[threadIdx.x] = my_fresh;
    __syncthreads();
    for (int32_t w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int32_t)threadIdx.x < w) sh_n[threadIdx.x] += sh_n[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && (a.full || a.admit))
        g->quiet = (a.full && !a.admit && !a.batch_avg && sh_n[0] == 0) ? 1 : 0;

    // compaction plan (full evaluations, stopping tests, and admissions that ask
    // for one): live prefix [0, n_run)
    if (a.admit && !a.admit_plan) {
        if (threadIdx.x == 0) {
            g->n_retire = 0;
            g->n_move = 0;
            g->n_fresh = 0;
            g->n_cols_next = nc;
        }
    } else if (a.full || a.stop_only || a.admit) {
        for (int32_t s = threadIdx.x; s < nc; s += blockDim.x) sh_flags[s] = a.sl.key[s].flags;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t nr = 0, nm = 0, nf = 0;
            int32_t mover = n_run;   // scan for running slots at or beyond n_run
            for (int32_t s = 0; s < nc; ++s) {
                const int32_t fl = sh_flags[s];
                if (!(fl & SLOT_RETIRE)) {
                    // restarted LPs that keep their slot; those beyond n_run restart
                    // as they move (at an admission the flag of an LP restarted by the
                    // last full evaluation still waits for its residual evaluation,
                    // and that evaluation's plan already made z~ its anchor)
                    if ((fl & SLOT_ACTIVE) && (fl & SLOT_FRESH) && s < n_run && !a.admit)
                        a.fresh[nf++] = s;
                    continue;
                }
                const int32_t lp = a.sl.lp[s];
                const int32_t kl = a.ctl[lp].k_last;
                RetireEntry re;
                re.slot = s;
                re.lp = lp;
                re.kp2 = kl + 2;
                re.src = -1;
                re.a = double(kl + 1) / double(kl + 2);
                re.src_fresh = 0;
                re.pad = 0;
                if (s < n_run) {
                    // the running slots at or beyond n_run are exactly as many as the
                    // stopped slots below it; the bound only guards that count
                    while (mover < nc && !(sh_flags[mover] & SLOT_ACTIVE)) ++mover;
                    if (mover < nc) {
                        a.moves[nm].src = mover;
                        a.moves[nm].dst = s;
                        nm += 1;
                        re.src = mover;
                        re.src_fresh = (!a.admit && (sh_flags[mover] & SLOT_FRESH)) ? 1 : 0;
                        ++mover;
                    }
                }
                a.retire[nr++] = re;
            }
            g->n_retire = nr;
            g->n_move = nm;
            g->n_fresh = nf;
            g->n_cols_next = n_run;
        }
    }
    if (threadIdx.x == 0) {
        g->n_active = n_run;
        if (a.advance) g->t0 += a.block;
    }
}

// ---------------------------------------------------------------------------
// Plan of a full evaluation (Section 4, restarts; Section 5, per-LP stop and
// compaction), one launch:
//   - restarted LPs that stay in place: anchor and dual iterate become z~
//     (X0 = Xt, Y0 = Y = Yt; Xbar needs no update, since at k = 0 the primal
//     step reads the anchor only);
//   - stopped LPs: z~ and the last Halpern iterate are copied to the LP-major
//     result blocks;
//   - a running LP beyond the new column count moves into the slot of a
//     stopped one, after that slot's results are copied out (the same thread
//     reads the old column and then writes the new one), taking a restart
//     decided at this evaluation on the way.
// A workgroup owns TR consecutive rows (x rows first, then y rows) and takes
// the plan entries 64 at a time; its threads take the (entry, row) pairs of
// the tile, entries fastest, so a few retiring LPs still occupy every thread
// and issue the tile's loads at once.  Reads and writes of the row-major
// blocks run along slots, and the entries of one row tile share its lines, so
// one workgroup walking all of them reads each line once; the results pass
// through LDS so that each LP's TR values of a result block are written as one
// contiguous segment.  TR * sizeof(T) = 256 bytes.
// ---------------------------------------------------------------------------
template <typename T>
struct Blocks8 {
    T* b[8];
};

template <typename T>
__global__ __launch_bounds__(256) void k_compact(int32_t n, int32_t m, int32_t ld, Blocks8<T> B,
                                                 Blocks8<T> R, const RetireEntry* retire,
                                                 const MoveEntry* moves, const int32_t* fresh,
                                                 Slots sl, Globals* g) {
    constexpr int TR = 256 / (int)sizeof(T);
    __shared__ T res_t[64][TR + 1];   // z~ of each entry's LP, rows of the tile
    __shared__ T res_h[64][TR + 1];   // its last Halpern iterate
    __shared__ RetireEntry ent[64];   // the entries of the current chunk
    const int32_t nr = g->n_retire, nf = g->n_fresh, nm = g->n_move;
    const int32_t tiles_x = (n + TR - 1) / TR;
    const bool xside = (int32_t)blockIdx.x < tiles_x;
    const int32_t r0 = (xside ? (int32_t)blockIdx.x : (int32_t)blockIdx.x - tiles_x) * TR;
    const int32_t rows = xside ? n : m;
    const int32_t rcount = min(TR, rows - r0);

    // (slot, row) pairs of the restarted slots that stay in place, slots fastest
    for (int32_t idx = threadIdx.x; idx < nf * rcount; idx += 256) {
        const int32_t q = idx % nf, rr = idx / nf;
        const size_t e = (size_t)(r0 + rr) * ld + fresh[q];
        if (xside) {
            B.b[1][e] = B.b[2][e];
        } else {
            const T v = B.b[6][e];
            B.b[5][e] = v;
            B.b[4][e] = v;
        }
    }
    for (int32_t q0 = 0; q0 < nr; q0 += 64) {
        const int32_t nq = min(64, nr - q0);
        if ((int32_t)threadIdx.x < nq) ent[threadIdx.x] = retire[q0 + threadIdx.x];
        __syncthreads();
        // (entry, row) pairs of the tile, entries fastest; the thread of a pair
        // reads the entry's old column at that row and then writes the new one
        for (int32_t idx = threadIdx.x; idx < nq * rcount; idx += 256) {
            const int32_t qq = idx % nq, rr = idx / nq;
            const RetireEntry& re = ent[qq];
            const size_t base = (size_t)(r0 + rr) * ld;
            const size_t e = base + re.slot;
            if (xside) {
                const T xb = B.b[0][e], x0 = B.b[1][e], xt = B.b[2][e];
                res_t[qq][rr] = xt;
                res_h[qq][rr] = halpern_last<T>(re.a, re.kp2, xb, x0);
            } else {
                res_t[qq][rr] = B.b[6][e];   // y~
                res_h[qq][rr] = B.b[4][e];   // Halpern iterate y^{k+1}
            }
            if (re.src >= 0) {
                // a moving LP takes its iterate and anchor along (z~ as both
                // when it restarted at this evaluation); its z~ and
                // displacement are written again by the iteration before any
                // later evaluation reads them
                const size_t f = base + re.src;
                if (xside) {
                    const T v0 = B.b[0][f];
                    const T v1 = re.src_fresh ? B.b[2][f] : B.b[1][f];
                    B.b[0][e] = v0;
                    B.b[1][e] = v1;
                } else {
                    const T v4 = re.src_fresh ? B.b[6][f] : B.b[4][f];
                    const T v5 = re.src_fresh ? v4 : B.b[5][f];
                    B.b[4][e] = v4;
                    B.b[5][e] = v5;
                }
            }
        }
        __syncthreads();
        // transposed write: each entry's rows of the tile as one contiguous run
        T* rt = xside ? R.b[0] : R.b[2];
        T* rh = xside ? R.b[1] : R.b[3];
        for (int32_t idx = threadIdx.x; idx < nq * TR; idx += 256) {
            const int32_t qq = idx / TR, rr = idx % TR;
            if (rr >= rcount) continue;
            const int32_t lp = ent[qq].lp;
            const size_t o = (size_t)lp * rows + r0 + rr;
            rt[o] = res_t[qq][rr];
            rh[o] = res_h[qq][rr];
        }
        __syncthreads();   // the next entries reuse the LDS rows
    }
    if (blockIdx.x == 0) {
        // slot state of the moved LPs; no other workgroup of this launch reads it
        for (int32_t k = threadIdx.x; k < nm; k += blockDim.x) {
            const MoveEntry mv = moves[k];
            sl.key[mv.dst] = sl.key[mv.src];
            sl.tau[mv.dst] = sl.tau[mv.src];
            sl.sigma[mv.dst] = sl.sigma[mv.src];
            sl.dval[mv.dst] = sl.dval[mv.src];
            sl.t_start[mv.dst] = sl.t_start[mv.src];
            sl.lp[mv.dst] = sl.lp[mv.src];
        }
        __syncthreads();
        if (threadIdx.x == 0) g->n_cols = g->n_cols_next;
    }
}

// ---------------------------------------------------------------------------
// Persistent tail (Section 5: the LPs still running once most of a batch has
// stopped).  One workgroup of TAIL_THREADS threads owns one running LP and
// runs its remaining iterations, evaluations, restarts and stop inside one
// launch, so a narrow tail pays no launch boundaries.  It follows the batched
// schedule exactly: blocks of C iterations from the next block base t0; an
// evaluation of a fresh restart cycle (or of a last iteration) after the first
// iteration of a block, a full evaluation after the last.  The LP's column is
// copied to contiguous vectors first (the two that the products gather, X-bar
// and Y, into LDS).  One CU streams the whole matrix every iteration, so the
// tail pays only for small matrices (a few thousand nonzeros).  Every quantity is computed as the batched kernels
// compute it -- the same row products in CSR order, the same coordinate
// updates, the same evaluation chains of pw rows per wave, panel sums
// ((c0 + c1) + c2) + c3, lane-strided panel sums and butterfly, and the same
// control -- so the LP's results are those of the batched path, bit for bit.
// ---------------------------------------------------------------------------
template <typename T>
struct TailVec {
    T *xb, *x0, *xt, *dx, *y, *y0, *yt, *dy;
};

// One side of an evaluation: chain sums (chain c = 4 panel + wave, rows
// [c pw, (c + 1) pw)), panel values, then the 64-lane reduction of term q
// into sums[q].  Waves take 64 / pw chains at once when pw < 64.
template <typename T>
__device__ void tail_eval_side(const TailArgs<T>& a, const TailVec<T>& v, int32_t s,
                               int32_t varkind, bool xside, double* chain, double* panel,
                               double* sums, double (*terms)[NTERM + 1], int lane, int wave,
                               int tid) {
    constexpr int NW = TAIL_THREADS / 64;
    const int32_t np = xside ? a.npx : a.npy;
    const int32_t pw = xside ? a.pw_x : a.pw_y;
    const int32_t rows = xside ? a.n : a.m;
    const int32_t nchains = 4 * np;
    const int32_t per = pw < 64 ? pw : 64;        // rows of one chain in one trip
    const int32_t G = 64 / per;                   // chains of a wave in one trip
    const int32_t trips = pw < 64 ? 1 : pw / 64;
    const int32_t npair = G * NTERM;
    for (int32_t cb = 0; cb < nchains; cb += NW * G) {
        const int32_t c0 = cb + wave * G;
        double acc[3] = {0.0, 0.0, 0.0};          // pairs lane, lane + 64, lane + 128
        for (int32_t tr = 0; tr < trips; ++tr) {
            const int32_t c = c0 + lane / per;
            const int32_t i = c * pw + tr * 64 + lane % per;
            const int32_t r1 = min((c + 1) * pw, rows);
            if (c < nchains && i < r1) {
                double tq[NTERM];
                if (xside) {
                    const XRow r{(double)v.xt[i], (double)v.dx[i], (double)v.x0[i], a.c[i], a.xl[i],
                                 a.xu[i]};
                    double g = 0.0, h = 0.0, pdy = 0.0;
                    for (int32_t k = a.t_rp[i]; k < a.t_rp[i + 1]; ++k) {
                        const int32_t j = a.t_ci[k];
                        const double w = (double)a.t_v[k];
                        const double yv = (double)v.yt[j], dv = (double)v.dy[j];
                        g = fma(w, yv, g);
                        h = fma(w, dv, h);
                        pdy = fma(w, barrier(dv, a.rl[j], a.ru[j]), pdy);
                    }
                    finish_xrow(r, g, h, pdy, varkind, a.sl.dval, s, i, tq);
                } else {
                    const YRow r{(double)v.yt[i], (double)v.dy[i], (double)v.y0[i], a.rl[i], a.ru[i]};
                    double ax = 0.0, adx = 0.0;
                    for (int32_t k = a.a_rp[i]; k < a.a_rp[i + 1]; ++k) {
                        const int32_t j = a.a_ci[k];
                        const double w = (double)a.a_v[k];
                        ax = fma(w, (double)v.xt[j], ax);
                        adx = fma(w, (double)v.dx[j], adx);
                    }
                    finish_yrow(r, ax, adx, tq);
                }
#pragma unroll
                for (int q = 0; q < NTERM; ++q) terms[wave * 64 + lane][q] = tq[q];
            }
            __syncthreads();
#pragma unroll
            for (int pi = 0; pi < 3; ++pi) {
                const int32_t pair = lane + 64 * pi;
                if (pair < npair) {
                    const int32_t cl = pair / NTERM, q = pair % NTERM;
                    const int32_t c2 = c0 + cl;
                    if (c2 < nchains) {
                        const int32_t rb = c2 * pw + tr * 64;
                        const int32_t cnt = min(per, min((c2 + 1) * pw, rows) - rb);
                        for (int32_t jj = 0; jj < cnt; ++jj) acc[pi] += terms[wave * 64 + cl * per + jj][q];
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int pi = 0; pi < 3; ++pi) {
            const int32_t pair = lane + 64 * pi;
            if (pair < npair) {
                const int32_t c2 = c0 + pair / NTERM;
                if (c2 < nchains) chain[(size_t)c2 * NTERM + pair % NTERM] = acc[pi];
            }
        }
    }
    __syncthreads();
    // panel values, term-major: panel[q np + p]
    for (int32_t idx = tid; idx < np * NTERM; idx += TAIL_THREADS) {
        const int32_t p = idx / NTERM, q = idx % NTERM;
        const double* cc = chain + (size_t)4 * p * NTERM + q;
        panel[(size_t)q * np + p] = ((cc[0] + cc[NTERM]) + cc[2 * NTERM]) + cc[3 * NTERM];
    }
    __syncthreads();
    // term q: lane l adds panels l, l + 64, ... in order, then a butterfly
    for (int32_t q = wave; q < NTERM; q += NW) {
        double acc = 0.0;
        for (int32_t i = lane; i < np; i += 64) acc += panel[(size_t)q * np + i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) sums[q] = acc;
    }
    __syncthreads();
}

// One row's product with a vector held in LDS, in CSR order: the first eight
// entries from the 8-wide ELL copy (no wait for the row pointers), the rest of
// a longer row from the CSR arrays.  A thread takes TAIL_ROWS rows at a time
// and issues all of their ELL loads before the first gather, so that several
// rows' loads are in flight in each of the workgroup's few waves.
constexpr int TAIL_ROWS = 2;

template <typename T>
struct TailEll {
    int32_t j[8];
    T w[8];
};

template <typename T>
__device__ __forceinline__ void tail_ell_load(const int32_t* eci, const T* ev, int32_t i,
                                              TailEll<T>& r) {
    const int4* q = reinterpret_cast<const int4*>(eci + (size_t)i * 8);
    const int4 j0 = q[0], j1 = q[1];
    r.j[0] = j0.x; r.j[1] = j0.y; r.j[2] = j0.z; r.j[3] = j0.w;
    r.j[4] = j1.x; r.j[5] = j1.y; r.j[6] = j1.z; r.j[7] = j1.w;
    HeadVals<T, 8>::load(ev + (size_t)i * 8, r.w);
}

// The ELL part: padding entries (index -1) leave the sum as it is.
template <typename T>
__device__ __forceinline__ T tail_ell_dot(const TailEll<T>& r, const T* sv) {
    T acc = T(0);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const T g = sv[r.j[u] < 0 ? 0 : r.j[u]];
        const T f = fma(r.w[u], g, acc);
        acc = r.j[u] >= 0 ? f : acc;
    }
    return acc;
}

// Entries past the first eight, in CSR order.
template <typename T>
__device__ __forceinline__ T tail_rest(const TailEll<T>& r, const int32_t* rp, const int32_t* ci,
                                       const T* av, int32_t i, const T* sv, T acc) {
    if (r.j[7] >= 0) {
        const int32_t ke = rp[i + 1];
        for (int32_t k = rp[i] + 8; k < ke; ++k) acc = fma(av[k], sv[ci[k]], acc);
    }
    return acc;
}

template <typename T>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(TailArgs<T> a) {
    __shared__ double terms[TAIL_THREADS][NTERM + 1];
    __shared__ int32_t sh_stop;
    extern __shared__ double tail_lds[];   // Xbar (n) and Y (m), the vectors the products gather
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tid = threadIdx.x;
    const int32_t s = blockIdx.x;
    if (s >= a.ncols) return;
    SlotKey* keyp = a.sl.key + s;
    if (!(keyp->flags & SLOT_ACTIVE)) return;
    const int32_t n = a.n, m = a.m, ld = a.ld;
    TailVec<T> v;
    T* const wbase = a.work + (size_t)s * (4 * (size_t)n + 4 * (size_t)m);
    v.xb = reinterpret_cast<T*>(tail_lds);
    v.x0 = wbase + n;
    v.xt = v.x0 + n;
    v.dx = v.xt + n;
    v.y = v.xb + n;
    v.y0 = v.dx + n + m;
    v.yt = v.y0 + m;
    v.dy = v.yt + m;
    for (int32_t i = tid; i < n; i += TAIL_THREADS) {
        const size_t e = (size_t)i * ld + s;
        v.xb[i] = a.blk[0][e];
        v.x0[i] = a.blk[1][e];
        v.xt[i] = a.blk[2][e];
        v.dx[i] = a.blk[3][e];
    }
    for (int32_t i = tid; i < m; i += TAIL_THREADS) {
        const size_t e = (size_t)i * ld + s;
        v.y[i] = a.blk[4][e];
        v.y0[i] = a.blk[5][e];
        v.yt[i] = a.blk[6][e];
        v.dy[i] = a.blk[7][e];
    }
    double* ws = a.wsum + (size_t)s * tail_sum_doubles(a.npx, a.npy);
    double* chain_x = ws;
    double* chain_y = chain_x + (size_t)4 * a.npx * NTERM;
    double* panel_x = chain_y + (size_t)4 * a.npy * NTERM;
    double* panel_y = panel_x + (size_t)a.npx * NTERM;
    double* sums = panel_y + (size_t)a.npy * NTERM;   // x side [0, NTERM), y side [NTERM, 2 NTERM)
    const double eta = a.g->eta;
    int32_t t0 = a.g->t0;
    const int32_t lp = a.sl.lp[s];
    __syncthreads();
    for (;;) {
        bool stopped = false;
        for (int32_t it = 1; it <= a.C && !stopped; ++it) {
            const int32_t t = t0 + it;
            const SlotKey key = *keyp;
            const int32_t k = t - key.t_anchor;
            const bool stop_it = a.S > 0 && it % a.S == 0 && it != a.C;
            if ((key.flags & SLOT_ACTIVE) && t <= key.t_end) {
                // the evaluation after this iteration reads z~ and the displacement
                const bool keep = t == key.t_end || it == a.C || (it == 1 && k == 0) || stop_it;
                const T tau = T(a.sl.tau[s]);
                for (int32_t i0 = tid; i0 < n; i0 += TAIL_ROWS * TAIL_THREADS) {
                    TailEll<T> e[TAIL_ROWS];
                    T acc[TAIL_ROWS], x0v[TAIL_ROWS];
                    double cv[TAIL_ROWS], lv[TAIL_ROWS], hv[TAIL_ROWS];
#pragma unroll
                    for (int r = 0; r < TAIL_ROWS; ++r) {
                        const int32_t i = min(i0 + r * TAIL_THREADS, n - 1);   // past n: row n-1, unused
                        tail_ell_load<T>(a.t_e8ci, a.t_e8v, i, e[r]);
                        cv[r] = a.c[i];
                        lv[r] = a.xl[i];
                        hv[r] = a.xu[i];
                        x0v[r] = v.x0[i];
                    }
#pragma unroll
                    for (int r = 0; r < TAIL_ROWS; ++r) acc[r] = tail_ell_dot<T>(e[r], v.y);
#pragma unroll
                    for (int r = 0; r < TAIL_ROWS; ++r) {
                        const int32_t i = i0 + r * TAIL_THREADS;
                        if (i < n) {
                            const T pr = tail_rest<T>(e[r], a.t_rp, a.t_ci, a.t_v, i, v.y, acc[r]);
                            const VarData d = var_data(key.varkind, a.sl.dval, s, i, cv[r], lv[r], hv[r]);
                            T xk, xt, xbar;
                            primal_point<T>(k, v.xb[i], x0v[r], tau, d.c, d.lo, d.hi, pr, xk, xt, xbar);
                            v.xb[i] = xbar;
                            if (keep) {
                                v.xt[i] = xt;
                                v.dx[i] = xt - xk;
                            }
                        }
                    }
                }
                __syncthreads();
                const T sg = T(a.sl.sigma[s]);
                const T wa = T(halpern_a(k)), wb = T(k + 2);
                for (int32_t i0 = tid; i0 < m; i0 += TAIL_ROWS * TAIL_THREADS) {
                    TailEll<T> e[TAIL_ROWS];
                    T acc[TAIL_ROWS], y0v[TAIL_ROWS];
                    double lv[TAIL_ROWS], hv[TAIL_ROWS];
#pragma unroll
                    for (int r = 0; r < TAIL_ROWS; ++r) {
                        const int32_t i = min(i0 + r * TAIL_THREADS, m - 1);   // past m: row m-1, unused
                        tail_ell_load<T>(a.a_e8ci, a.a_e8v, i, e[r]);
                        lv[r] = a.rl[i];
                        hv[r] = a.ru[i];
                        y0v[r] = v.y0[i];
                    }
#pragma unroll
                    for (int r = 0; r < TAIL_ROWS; ++r) acc[r] = tail_ell_dot<T>(e[r], v.xb);
#pragma unroll
                    for (int r = 0; r < TAIL_ROWS; ++r) {
                        const int32_t i = i0 + r * TAIL_THREADS;
                        if (i < m) {
                            const T pr = tail_rest<T>(e[r], a.a_rp, a.a_ci, a.a_v, i, v.xb, acc[r]);
                            const T yk = v.y[i];
                            T yt, yn;
                            dual_point<T>(yk, y0v[r], sg, wa, wb, T(lv[r]), T(hv[r]), pr, yt, yn);
                            v.y[i] = yn;
                            if (keep) {
                                v.yt[i] = yt;
                                v.dy[i] = yt - yk;
                            }
                        }
                    }
                }
                __syncthreads();
            }
            if (it != 1 && it != a.C && !stop_it) continue;
            const bool full = it == a.C;
            // between full evaluations only a fresh cycle, a stopping test or a last
            // iteration is evaluated
            if (!(full || stop_it || t == key.t_anchor || t >= key.t_end)) continue;
            tail_eval_side<T>(a, v, s, key.varkind, true, chain_x, panel_x, sums, terms, lane, wave, tid);
            tail_eval_side<T>(a, v, s, key.varkind, false, chain_y, panel_y, sums + NTERM, terms, lane,
                              wave, tid);
            if (tid == 0) {
                double r = 0.0;
                bool rh = false;
                sh_stop = control_slot(a.ca, full, stop_it, s, *keyp, a.ctl[lp],
                                       a.rlog + (size_t)lp * RESTART_LOG, sums, sums + NTERM, 1, t,
                                       eta, true, &r, &rh);
            }
            __syncthreads();
            stopped = sh_stop != 0;
            if (full && !stopped && (keyp->flags & SLOT_FRESH)) {
                // restart: anchor and dual iterate become z~ (Section 4)
                for (int32_t i = tid; i < n; i += TAIL_THREADS) v.x0[i] = v.xt[i];
                for (int32_t i = tid; i < m; i += TAIL_THREADS) {
                    const T yt = v.yt[i];
                    v.y0[i] = yt;
                    v.y[i] = yt;
                }
                __syncthreads();
            }
        }
        if (stopped) break;
        t0 += a.C;
    }
    // results: z~ and the last Halpern iterate (as the compaction copies them)
    const int32_t kl = a.ctl[lp].k_last;
    const double ha = double(kl + 1) / double(kl + 2);
    for (int32_t i = tid; i < n; i += TAIL_THREADS) {
        a.res[0][(size_t)lp * n + i] = v.xt[i];
        a.res[1][(size_t)lp * n + i] = halpern_last<T>(ha, kl + 2, v.xb[i], v.x0[i]);
    }
    for (int32_t i = tid; i < m; i += TAIL_THREADS) {
        a.res[2][(size_t)lp * m + i] = v.yt[i];
        a.res[3][(size_t)lp * m + i] = v.y[i];
    }
}

// ---------------------------------------------------------------------------
// batch set-up
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_init_blocks(int32_t n, int32_t m, int32_t ld, int32_t ncols, Slots sl,
                              const double* xl, const double* xu, const double* xw,
                              const double* yw, int32_t mode, T* Xbar, T* X0, T* Y, T* Y0) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nx = (int64_t)n * ld, ny = (int64_t)m * ld;
    if (idx < nx) {
        const int32_t i = (int32_t)(idx / ld), s = (int32_t)(idx % ld);
        T x = T(0);
        if (s < ncols) {
            const VarData d = var_data(sl.key[s].varkind, sl.dval, s, i, 0.0, xl[i], xu[i]);
            double w0 = 0.0;
            if (mode == PDLPB_WARM_SHARED) w0 = xw[i];
            else if (mode == PDLPB_WARM_PER_LP) w0 = xw[(size_t)sl.lp[s] * n + i];
            x = T(clampd(w0, d.lo, d.hi));
        }
        Xbar[idx] = x;
        X0[idx] = x;
    } else if (idx < nx + ny) {
        const int64_t e = idx - nx;
        const int32_t i = (int32_t)(e / ld), s = (int32_t)(e % ld);
        T y = T(0);
        if (s < ncols) {
            if (mode == PDLPB_WARM_SHARED) y = T(yw[i]);
            else if (mode == PDLPB_WARM_PER_LP) y = T(yw[(size_t)sl.lp[s] * m + i]);
        }
        Y[e] = y;
        Y0[e] = y;
    }
}

__global__ void k_begin_solve(Slots sl, SlotCtl* ctl, int32_t ncols, int32_t max_iters, Globals* g,
                              double tol) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ncols) {
        sl.t_start[s] = 0;
        sl.key[s].t_anchor = 0;
        sl.key[s].t_end = max_iters - 1;
        SlotCtl& cl = ctl[sl.lp[s]];
        cl.status = PDLPB_STATUS_RUNNING;
        cl.restarts = 0;
        cl.r_prev = -1.0;
        cl.tol = tol;
    }
    if (s == 0) {
        g->t0 = 0;
        g->tol = tol;
        g->batch_k0 = 0;
        g->r_prev = -1.0;
        g->n_active = ncols;
        g->n_cols = ncols;
        g->n_retire = 0;
        g->n_move = 0;
        g->n_fresh = 0;
        g->n_cols_next = ncols;
        g->quiet = 0;
    }
}

template <typename T>
__global__ void k_init_columns(int32_t n, int32_t m, int32_t ld, int32_t c0, int32_t cnt, Slots sl,
                               const double* xl, const double* xu, const double* xw,
                               const double* yw, int32_t mode, Blocks8<T> B) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nx = (int64_t)n * cnt, ny = (int64_t)m * cnt;
    if (idx < nx) {
        const int32_t i = (int32_t)(idx / cnt), s = c0 + (int32_t)(idx % cnt);
        const VarData d = var_data(sl.key[s].varkind, sl.dval, s, i, 0.0, xl[i], xu[i]);
        const T x = T(clampd(mode == PDLPB_WARM_BASE ? xw[i] : 0.0, d.lo, d.hi));
        const size_t e = (size_t)i * ld + s;
        B.b[0][e] = x;
        B.b[1][e] = x;
        B.b[2][e] = x;
        B.b[3][e] = T(0);
    } else if (idx < nx + ny) {
        const int64_t q = idx - nx;
        const int32_t i = (int32_t)(q / cnt), s = c0 + (int32_t)(q % cnt);
        // objective changes start from the base primal point with y = 0
        const bool objective = (sl.key[s].varkind >> 28) == PDLPB_OBJ_UNIT;
        const T y = (mode == PDLPB_WARM_BASE && !objective) ? T(yw[i]) : T(0);
        const size_t e = (size_t)i * ld + s;
        B.b[4][e] = y;
        B.b[5][e] = y;
        B.b[6][e] = y;
        B.b[7][e] = T(0);
    }
}

__global__ void k_admit(SlotCtl* ctl, const int32_t* rows, const SlotCtl* src, int32_t cnt,
                        Globals* g, int32_t n_cols) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) ctl[rows[i]] = src[i];
    if (i == 0) {
        g->n_cols = n_cols;
        g->quiet = 0;
    }
}

// v[k] *= d[k % period] (or /=): maps LP-major blocks and shared vectors
// between the caller's coordinates and the scaled LP's
__global__ void k_rescale(double* v, const double* d, int64_t count, int32_t period,
                          int32_t divide) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) {
        const double f = d[k % period];
        v[k] = divide ? v[k] / f : v[k] * f;
    }
}

__global__ void k_widen(const float* src, int64_t count, double* dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = (double)src[i];
}

// ---------------------------------------------------------------------------
// power iteration helpers (float64)
// ---------------------------------------------------------------------------
__global__ void k_spmv(const int32_t* rp, const int32_t* ci, const double* v, int32_t rows,
                       const double* x, double* y) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    double acc = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) acc = fma(v[k], x[ci[k]], acc);
    y[i] = acc;
}

constexpr int NORM_BLOCKS = 1024;

__global__ __launch_bounds__(256) void k_norm_partial(const double* x, int32_t len, double* part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * 256)
        acc = fma(x[i], x[i], acc);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_norm_final(const double* part, int32_t np, double* out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int32_t i = threadIdx.x; i < np; i += 256) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_scale(double* x, int32_t len, const double* nrm2sq) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) x[i] = x[i] / sqrt(*nrm2sq);
}

__global__ void k_fill(double* x, int32_t len, double v) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) x[i] = v;
}

// ---------------------------------------------------------------------------
// Shared start (Section 5: the LPs of a strong-branching or bound-tightening
// batch each change one variable of a common LP).  When every running LP
// starts from the same point, with the same step sizes as the other LPs of its
// base LP, T(z^0) of an LP
// differs from that of its base LP -- the common LP, or for an objective
// change the common LP with objective 0 -- only at its variable v (x^0 for a
// bound change; x~, x-bar, dx) and at the rows of A through v (y~, y^1, dy).
// Its evaluation terms at t = 0 then differ only on x rows that are v or
// share a row of A with v and on y rows through v, and a chain of rows
// (evaluation panel unit) without such a row sums to its base LP's value.
// These kernels make the first iteration of each base LP once, of each LP
// only at those coordinates, the terms and chain sums of each base LP once,
// and each LP's chains only where it differs.  Products, coordinate updates,
// terms and sums are those of the step and evaluation kernels, in the same
// order, so every LP's panel sums are the bits k_eval computes from its
// blocks.  After the control pass the blocks are written only for the LPs
// that still run, at their slots after the compaction, and the stopped LPs'
// results go straight to the result blocks.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int32_t sp_class(const SharedArgs<T>& a, int32_t varkind) {
    return ((uint32_t)varkind >> 28) == (uint32_t)PDLPB_OBJ_UNIT ? a.cls_obj : a.cls_bound;
}
// delta key of base LP K (no variable)
template <typename T>
__device__ __forceinline__ int32_t sp_base_key(const SharedArgs<T>& a, int32_t K) {
    return VAR_NONE | (a.cls_kind[K] << 28);
}
// y^0 as the blocks hold it
template <typename T>
__device__ __forceinline__ T sp_y0(const SharedArgs<T>& a, int32_t r) {
    return a.yw ? T(a.yw[r]) : T(0);
}

// x^0 on the base box and, per base LP, x~, x-bar and dx of the first step:
// one thread per variable, (A'y^0)_i summed in CSR order from 0 as the primal
// step kernel sums it.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_primal(SharedArgs<T> a) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const double lo = a.xl[i], hi = a.xu[i];
    const T x0 = T(clampd(a.xw ? a.xw[i] : 0.0, lo, hi));
    T g = T(0);
    for (int32_t k = a.t_rp[i]; k < a.t_rp[i + 1]; ++k) g = fma(a.t_v[k], sp_y0(a, a.t_ci[k]), g);
    a.x0[i] = x0;
    for (int32_t K = 0; K < a.ncls; ++K) {
        const VarData d = var_data(sp_base_key(a, K), nullptr, 0, i, a.c[i], lo, hi);
        T xk, xt, xbar;
        primal_point<T>(0, T(0), x0, T(a.tau[K]), d.c, d.lo, d.hi, g, xk, xt, xbar);
        const size_t e = (size_t)K * a.n + i;
        a.xt[e] = xt;
        a.xbar[e] = xbar;
        a.dx[e] = xt - xk;
    }
}

// y^0 and, per base LP, y~, y^1 and dy of the first step: one thread per row.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_dual(SharedArgs<T> a) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.m) return;
    const T y0 = sp_y0(a, r);
    const T l = T(a.rl[r]), u = T(a.ru[r]);
    a.y0[r] = y0;
    for (int32_t K = 0; K < a.ncls; ++K) {
        const T* xb = a.xbar + (size_t)K * a.n;
        T v = T(0);
        for (int32_t k = a.a_rp[r]; k < a.a_rp[r + 1]; ++k) v = fma(a.a_v[k], xb[a.a_ci[k]], v);
        T yt, yn;
        dual_point<T>(y0, y0, T(a.sigma[K]), T(halpern_a(0)), T(2), l, u, v, yt, yn);
        const size_t e = (size_t)K * a.m + r;
        a.yt[e] = yt;
        a.yn[e] = yn;
        a.dy[e] = yt - y0;
    }
}

// The first step of each LP where it differs from its base LP: x at its
// variable v (its own box and objective entry), then y at the rows of A
// through v, whose products read its own x-bar at v.  One wave per slot.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_side(SharedArgs<T> a) {
    const int lane = threadIdx.x & 63;
    const int32_t s = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= a.nslots) return;
    const int32_t vk = a.sl.key[s].varkind;
    const int32_t v = vk & VAR_MASK;
    if (v == VAR_NONE) return;
    const int32_t K = sp_class(a, vk);
    T* side = a.side + (size_t)s * SP_SIDE;
    const VarData d0 = var_data(vk, a.sl.dval, s, v, 0.0, a.xl[v], a.xu[v]);
    const T x0 = T(clampd(a.xw ? a.xw[v] : 0.0, d0.lo, d0.hi));
    const int32_t kb = a.t_rp[v];
    const int32_t nv = min(a.t_rp[v + 1] - kb, SP_MAX_COL);
    T g = T(0);
    for (int32_t k = kb; k < a.t_rp[v + 1]; ++k) g = fma(a.t_v[k], sp_y0(a, a.t_ci[k]), g);
    const VarData d = var_data(vk, a.sl.dval, s, v, a.c[v], a.xl[v], a.xu[v]);
    T xk, xt, xbar;
    primal_point<T>(0, T(0), x0, T(a.tau[K]), d.c, d.lo, d.hi, g, xk, xt, xbar);
    if (lane == 0) {
        side[0] = x0;
        side[1] = xt;
        side[2] = xbar;
        side[3] = xt - xk;
    }
    const T* xb = a.xbar + (size_t)K * a.n;
    for (int32_t q = lane; q < nv; q += 64) {
        const int32_t r = a.t_ci[kb + q];
        T p = T(0);
        for (int32_t k = a.a_rp[r]; k < a.a_rp[r + 1]; ++k) {
            const int32_t j = a.a_ci[k];
            p = fma(a.a_v[k], j == v ? xbar : xb[j], p);
        }
        const T y0 = a.y0[r];
        T yt, yn;
        dual_point<T>(y0, y0, T(a.sigma[K]), T(halpern_a(0)), T(2), T(a.rl[r]), T(a.ru[r]), p, yt,
                      yn);
        T* o = side + 4 + 3 * q;
        o[0] = yt;
        o[1] = yn;
        o[2] = yt - y0;
    }
}

// Evaluation terms of x row i (x~, dx, x^0 at i given; y~ and dy at row r of A
// from yat) and of y row r (y~, dy, y^0 at r given; x~ and dx at column j from
// xat): the products in CSR order and the terms of k_eval.
template <typename T, typename YAt>
__device__ __forceinline__ void sp_xterms(const SharedArgs<T>& a, int32_t i, T xt, T dx, T x0,
                                          int32_t varkind, int32_t s, YAt yat, double* tv) {
    double g = 0.0, h = 0.0, pdy = 0.0;
    for (int32_t k = a.t_rp[i]; k < a.t_rp[i + 1]; ++k) {
        const int32_t r = a.t_ci[k];
        T yv, dv;
        yat(r, yv, dv);
        const double w = (double)a.t_v[k], d = (double)dv;
        g = fma(w, (double)yv, g);
        h = fma(w, d, h);
        pdy = fma(w, barrier_code(d, a.rcode[r]), pdy);
    }
    finish_xrow(XRowIn<T>{xt, dx, x0, a.c[i], a.xl[i], a.xu[i]}.wide(), g, h, pdy, varkind,
                a.sl.dval, s, i, tv);
}
template <typename T, typename XAt>
__device__ __forceinline__ void sp_yterms(const SharedArgs<T>& a, int32_t r, T yt, T dy, T y0,
                                          XAt xat, double* tv) {
    double ax = 0.0, adx = 0.0;
    for (int32_t k = a.a_rp[r]; k < a.a_rp[r + 1]; ++k) {
        T xv, dv;
        xat(a.a_ci[k], xv, dv);
        const double w = (double)a.a_v[k];
        ax = fma(w, (double)xv, ax);
        adx = fma(w, (double)dv, adx);
    }
    finish_yrow(YRowIn<T>{yt, dy, y0, a.rl[r], a.ru[r]}.wide(), ax, adx, tv);
}

// Terms of every row of each base LP, and its chain and panel sums: one
// workgroup per (panel, base LP) in the layout of k_eval_narrow (wave w sums
// rows [p0 + w pw, p0 + (w + 1) pw) in row order, 64 rows at a time, lane q
// adding term q; the panel sum is ((c0 + c1) + c2) + c3).
template <typename T>
__global__ __launch_bounds__(256) void k_sp_terms(SharedArgs<T> a) {
    __shared__ double terms[4][64][NTERM + 1];
    __shared__ double red[4][NTERM];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int32_t pidx = blockIdx.x, K = blockIdx.y;
    const int32_t np = a.npx + a.npy;
    const bool xside = pidx < a.npx;
    const int32_t panel = xside ? pidx : pidx - a.npx;
    const int32_t pw = xside ? a.pw_x : a.pw_y;
    const int32_t rows = xside ? a.n : a.m;
    const int32_t r0 = panel * 4 * pw + wave * pw;
    const int32_t r1 = min(r0 + pw, rows);
    const int32_t key = sp_base_key(a, K);
    const T* xt = a.xt + (size_t)K * a.n;
    const T* dx = a.dx + (size_t)K * a.n;
    const T* yt = a.yt + (size_t)K * a.m;
    const T* dy = a.dy + (size_t)K * a.m;
    double* rt = a.rt + (size_t)K * ((size_t)a.n + a.m) * NTERM;
    double acc = 0.0;
    for (int32_t off = 0; off < pw; off += 64) {
        const int32_t rb = r0 + off;
        const int32_t i = rb + lane;
        if (i < r1) {
            double tq[NTERM];
            if (xside) {
                sp_xterms(a, i, xt[i], dx[i], a.x0[i], key, 0,
                          [&](int32_t r, T& yv, T& dv) {
                              yv = yt[r];
                              dv = dy[r];
                          },
                          tq);
            } else {
                sp_yterms(a, i, yt[i], dy[i], a.y0[i],
                          [&](int32_t j, T& xv, T& dv) {
                              xv = xt[j];
                              dv = dx[j];
                          },
                          tq);
            }
            double* o = rt + (size_t)(xside ? i : a.n + i) * NTERM;
#pragma unroll
            for (int q = 0; q < NTERM; ++q) {
                o[q] = tq[q];
                terms[wave][lane][q] = tq[q];
            }
        }
        __syncthreads();
        if (lane < NTERM) {
            const int32_t cnt = min(64, r1 - rb);
            for (int32_t j = 0; j < cnt; ++j) acc += terms[wave][j][lane];
        }
        __syncthreads();
    }
    if (lane < NTERM) {
        red[wave][lane] = acc;
        a.bwave[(((size_t)K * np + pidx) * 4 + wave) * NTERM + lane] = acc;
    }
    __syncthreads();
    if (wave == 0 && lane < NTERM)
        a.bpanel[((size_t)K * np + pidx) * NTERM + lane] =
            ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Every running LP's panel sums set to its base LP's; k_sp_touched then
// replaces those of the panels the LP changes.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_bcast(SharedArgs<T> a) {
    const int32_t pidx = blockIdx.x;
    const int32_t s = blockIdx.y * 256 + threadIdx.x;
    if (s >= a.nslots) return;
    const int32_t K = sp_class(a, a.sl.key[s].varkind);
    const bool xside = pidx < a.npx;
    double* out = (xside ? a.part_x + (size_t)pidx * NTERM * a.ld
                         : a.part_y + (size_t)(pidx - a.npx) * NTERM * a.ld) + s;
    const double* bp = a.bpanel + ((size_t)K * (a.npx + a.npy) + pidx) * NTERM;
#pragma unroll
    for (int q = 0; q < NTERM; ++q) out[(size_t)q * a.ld] = bp[q];
}

constexpr int SP_SPLIT = 4;   // workgroups per LP in k_sp_touched

// Panel sums of one LP on the panels it changes: the x panels of v and of every
// column of the rows of A through v, the y panels of those rows.  SP_SPLIT
// one-wave workgroups per LP take its panels in turn.  A chain of rows with
// no row the LP changes takes its base LP's sum; any other chain is summed
// again in row order, from the LP's own terms on the rows it changes and its
// base LP's terms elsewhere.
template <typename T>
__global__ __launch_bounds__(64) void k_sp_touched(SharedArgs<T> a) {
    __shared__ double terms[64][NTERM + 1];
    __shared__ int32_t rv[SP_MAX_COL];   // the rows of A through v
    __shared__ uint32_t bits[128];       // changed panels: x in words [0, 64), y in [64, 128)
    __shared__ uint16_t list[4096];      // ... in panel order, x first
    __shared__ int32_t nlist;
    const int lane = threadIdx.x;
    const int32_t s = blockIdx.x;
    const int32_t vk = a.sl.key[s].varkind;
    const int32_t v = vk & VAR_MASK;
    if (v == VAR_NONE) return;
    const int32_t K = sp_class(a, vk);
    const int32_t kb = a.t_rp[v];
    const int32_t nv = min(a.t_rp[v + 1] - kb, SP_MAX_COL);
    const T* side = a.side + (size_t)s * SP_SIDE;
    const T* bxt = a.xt + (size_t)K * a.n;
    const T* bdx = a.dx + (size_t)K * a.n;
    const T* byt = a.yt + (size_t)K * a.m;
    const T* bdy = a.dy + (size_t)K * a.m;
    const double* rt = a.rt + (size_t)K * ((size_t)a.n + a.m) * NTERM;
    const int32_t np = a.npx + a.npy;
    const int32_t px = 4 * a.pw_x, py = 4 * a.pw_y;
    for (int32_t w = lane; w < 128; w += 64) bits[w] = 0u;
    for (int32_t q = lane; q < nv; q += 64) rv[q] = a.t_ci[kb + q];
    __syncthreads();
    if (lane == 0) atomicOr(&bits[(v / px) >> 5], 1u << ((v / px) & 31));
    for (int32_t q = 0; q < nv; ++q) {
        const int32_t r = rv[q];
        if (lane == 0) atomicOr(&bits[64 + ((r / py) >> 5)], 1u << ((r / py) & 31));
        for (int32_t k = a.a_rp[r] + lane; k < a.a_rp[r + 1]; k += 64) {
            const int32_t p = a.a_ci[k] / px;
            atomicOr(&bits[p >> 5], 1u << (p & 31));
        }
    }
    __syncthreads();
    if (lane == 0) {
        int32_t cnt = 0;
        for (int32_t w = 0; w < 128; ++w) {
            uint32_t b = bits[w];
            while (b) {
                const int32_t bit = __ffs(b) - 1;
                b &= b - 1;
                list[cnt++] = (uint16_t)(w < 64 ? w * 32 + bit : a.npx + (w - 64) * 32 + bit);
            }
        }
        nlist = cnt;
    }
    __syncthreads();
    const int32_t total = nlist;
    // the LP's y~, dy at row r of A and x~, dx at column j
    auto yat = [&](int32_t r, T& yv, T& dv) {
        for (int32_t q = 0; q < nv; ++q)
            if (rv[q] == r) {
                yv = side[4 + 3 * q];
                dv = side[4 + 3 * q + 2];
                return;
            }
        yv = byt[r];
        dv = bdy[r];
    };
    auto xat = [&](int32_t j, T& xv, T& dv) {
        if (j == v) {
            xv = side[1];
            dv = side[3];
        } else {
            xv = bxt[j];
            dv = bdx[j];
        }
    };
    // evaluation row i of one side reads a coordinate the LP changes
    auto changed = [&](bool xside, int32_t i) -> bool {
        if (xside) {
            if (i == v) return true;
            for (int32_t k = a.t_rp[i]; k < a.t_rp[i + 1]; ++k) {
                const int32_t r = a.t_ci[k];
                for (int32_t q = 0; q < nv; ++q)
                    if (rv[q] == r) return true;
            }
            return false;
        }
        for (int32_t q = 0; q < nv; ++q)
            if (rv[q] == i) return true;
        return false;
    };
    for (int32_t li = blockIdx.y; li < total; li += SP_SPLIT) {
        const int32_t pidx = list[li];
        const bool xside = pidx < a.npx;
        const int32_t panel = xside ? pidx : pidx - a.npx;
        const int32_t pw = xside ? a.pw_x : a.pw_y;
        const int32_t rows = xside ? a.n : a.m;
        double sum[4];
        for (int u = 0; u < 4; ++u) {
            const int32_t r0 = panel * 4 * pw + u * pw;
            const int32_t r1 = min(r0 + pw, rows);
            bool mine = false;
            for (int32_t off = 0; off < pw; off += 64) {
                const int32_t i = r0 + off + lane;
                if (i < r1 && changed(xside, i)) mine = true;
            }
            double acc = 0.0;
            if (!__syncthreads_or(mine)) {
                if (lane < NTERM) acc = a.bwave[(((size_t)K * np + pidx) * 4 + u) * NTERM + lane];
            } else {
                for (int32_t off = 0; off < pw; off += 64) {
                    const int32_t rb = r0 + off;
                    const int32_t i = rb + lane;
                    if (i < r1) {
                        double tq[NTERM];
                        if (!changed(xside, i)) {
                            const double* o = rt + (size_t)(xside ? i : a.n + i) * NTERM;
#pragma unroll
                            for (int q = 0; q < NTERM; ++q) tq[q] = o[q];
                        } else if (xside) {
                            const bool at_v = i == v;
                            sp_xterms(a, i, at_v ? side[1] : bxt[i], at_v ? side[3] : bdx[i],
                                      at_v ? side[0] : a.x0[i], vk, s, yat, tq);
                        } else {
                            int32_t q0 = 0;   // i is a row through v
                            while (rv[q0] != i) ++q0;
                            sp_yterms(a, i, side[4 + 3 * q0], side[4 + 3 * q0 + 2], a.y0[i], xat, tq);
                        }
#pragma unroll
                        for (int q = 0; q < NTERM; ++q) terms[lane][q] = tq[q];
                    }
                    __syncthreads();
                    if (lane < NTERM) {
                        const int32_t cnt = min(64, r1 - rb);
                        for (int32_t j = 0; j < cnt; ++j) acc += terms[j][lane];
                    }
                    __syncthreads();
                }
            }
            sum[u] = acc;
        }
        if (lane < NTERM) {
            double* out = (xside ? a.part_x : a.part_y) + (size_t)panel * NTERM * a.ld + s;
            out[(size_t)lane * a.ld] = ((sum[0] + sum[1]) + sum[2]) + sum[3];
        }
    }
}

// Live columns after the control pass: column e < n_cols_next holds the LP of
// slot map[e] (its own, or the one the plan moves into it), of base LP
// map[nslots + e].
template <typename T>
__global__ __launch_bounds__(1024) void k_sp_map(SharedArgs<T> a) {
    const int32_t nc = a.g->n_cols_next, nm = a.g->n_move;
    for (int32_t e = threadIdx.x; e < nc; e += blockDim.x) a.map[e] = e;
    __syncthreads();
    for (int32_t k = threadIdx.x; k < nm; k += blockDim.x) a.map[a.moves[k].dst] = a.moves[k].src;
    __syncthreads();
    for (int32_t e = threadIdx.x; e < nc; e += blockDim.x)
        a.map[a.nslots + e] = sp_class(a, a.sl.key[a.map[e]].varkind);
}

// Xbar, X0 (x rows) and Y, Y0 (y rows) of the live columns from their base
// LPs; k_sp_patch writes each LP's own values over them.  A workgroup writes
// the live columns of one row at a time, a contiguous run per block.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_dense(SharedArgs<T> a) {
    const int32_t nc = a.g->n_cols_next;
    const int32_t total = a.n + a.m;
    for (int32_t row = blockIdx.x; row < total; row += gridDim.x) {
        for (int32_t e = threadIdx.x; e < nc; e += blockDim.x) {
            const int32_t K = a.map[a.nslots + e];
            if (row < a.n) {
                const size_t o = (size_t)row * a.ld + e;
                a.blk[0][o] = a.xbar[(size_t)K * a.n + row];
                a.blk[1][o] = a.x0[row];
            } else {
                const int32_t r = row - a.n;
                const size_t o = (size_t)r * a.ld + e;
                a.blk[4][o] = a.yn[(size_t)K * a.m + r];
                a.blk[5][o] = a.y0[r];
            }
        }
    }
}

// Results of the LPs stopped at t = 0 from their base LPs (x~, the Halpern
// iterate rebuilt from x-bar and x^0 as k_compact does, y~, y^1): one thread
// per row loads the row's base values once and writes them into every stopped
// LP's result rows, a workgroup writing 256 consecutive entries of one LP at a
// time.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_results(SharedArgs<T> a) {
    const int32_t nr = a.g->n_retire;
    const int32_t row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= a.n + a.m) return;
    const bool xside = row < a.n;
    const int32_t i = xside ? row : row - a.n;
    // per base LP K: x~ and x-bar (y~ and y^1) of this row
    const T* p0 = xside ? a.xt : a.yt;
    const T* p1 = xside ? a.xbar : a.yn;
    const size_t len = xside ? (size_t)a.n : (size_t)a.m;
    const T a0 = p0[i], a1 = p1[i];
    const T b0 = a.ncls > 1 ? p0[len + i] : T(0), b1 = a.ncls > 1 ? p1[len + i] : T(0);
    const T x0 = xside ? a.x0[i] : T(0);
    for (int32_t q = 0; q < nr; ++q) {
        const RetireEntry re = a.retire[q];
        const bool second = sp_class(a, a.sl.key[re.slot].varkind) == 1;
        const T v0 = second ? b0 : a0, v1 = second ? b1 : a1;
        const size_t lp = (size_t)re.lp;
        if (xside) {
            a.res[0][lp * a.n + i] = v0;
            a.res[1][lp * a.n + i] = halpern_last<T>(re.a, re.kp2, v1, x0);
        } else {
            a.res[2][lp * a.m + i] = v0;
            a.res[3][lp * a.m + i] = v1;
        }
    }
}

// Each LP's own values at its variable and the rows through it, over the base
// values k_sp_dense and k_sp_results wrote: items [0, nslots) are live
// columns, items [nslots, 2 nslots) plan entries of stopped LPs.  One wave per
// item.
template <typename T>
__global__ __launch_bounds__(256) void k_sp_patch(SharedArgs<T> a) {
    const int lane = threadIdx.x & 63;
    const int32_t item = blockIdx.x * 4 + (threadIdx.x >> 6);
    const bool live = item < a.nslots;
    int32_t f, e = 0;
    RetireEntry re{};
    if (live) {
        e = item;
        if (e >= a.g->n_cols_next) return;
        f = a.map[e];
    } else {
        const int32_t q = item - a.nslots;
        if (q >= a.nslots || q >= a.g->n_retire) return;
        re = a.retire[q];
        f = re.slot;
    }
    const int32_t v = a.sl.key[f].varkind & VAR_MASK;
    if (v == VAR_NONE) return;
    const T* side = a.side + (size_t)f * SP_SIDE;
    const int32_t kb = a.t_rp[v];
    const int32_t nv = min(a.t_rp[v + 1] - kb, SP_MAX_COL);
    if (live) {
        if (lane == 0) {
            a.blk[0][(size_t)v * a.ld + e] = side[2];
            a.blk[1][(size_t)v * a.ld + e] = side[0];
        }
        for (int32_t q = lane; q < nv; q += 64)
            a.blk[4][(size_t)a.t_ci[kb + q] * a.ld + e] = side[4 + 3 * q + 1];
    } else {
        const size_t lp = (size_t)re.lp;
        if (lane == 0) {
            a.res[0][lp * a.n + v] = side[1];
            a.res[1][lp * a.n + v] = halpern_last<T>(re.a, re.kp2, side[2], side[0]);
        }
        for (int32_t q = lane; q < nv; q += 64) {
            const int32_t r = a.t_ci[kb + q];
            a.res[2][lp * a.m + r] = side[4 + 3 * q];
            a.res[3][lp * a.m + r] = side[4 + 3 * q + 1];
        }
    }
}

// Slot state of the moved LPs and the new column count, after every kernel
// that reads the old slots.
__global__ __launch_bounds__(1024) void k_sp_finish(Slots sl, const MoveEntry* moves, Globals* g) {
    const int32_t nm = g->n_move;
    for (int32_t k = threadIdx.x; k < nm; k += blockDim.x) {
        const MoveEntry mv = moves[k];
        sl.key[mv.dst] = sl.key[mv.src];
        sl.tau[mv.dst] = sl.tau[mv.src];
        sl.sigma[mv.dst] = sl.sigma[mv.src];
        sl.dval[mv.dst] = sl.dval[mv.src];
        sl.t_start[mv.dst] = sl.t_start[mv.src];
        sl.lp[mv.dst] = sl.lp[mv.src];
    }
    __syncthreads();
    if (threadIdx.x == 0) g->n_cols = g->n_cols_next;
}

template <typename T, int G, int VEC, int EW, bool PRIMAL>
hipError_t launch_step_gve(const StepArgs<T>& a, hipStream_t s) {
    constexpr int RPW = 64 / G;
    const int rows_per_block = a.wpb * RPW;
    const uint32_t gy = (uint32_t)((a.ncols + G * VEC - 1) / (G * VEC));
    uint32_t gx = (uint32_t)((a.rows + rows_per_block - 1) / rows_per_block);
    if (a.max_blocks > 0 && gy > 0) {
        // at most max_blocks workgroups in all; their waves loop over the row groups
        const uint32_t cap = (uint32_t)max(1, a.max_blocks / (int32_t)gy);
        gx = min(gx, cap);
    }
    const dim3 grid(gx, gy);
    const dim3 block(64 * a.wpb);
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
    if (PRIMAL)
        hipLaunchKernelGGL((k_primal<T, G, VEC, EW>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_dual<T, G, VEC, EW>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <typename T, int G, int VEC, bool PRIMAL>
hipError_t launch_step_gv(const StepArgs<T>& a, hipStream_t s) {
    switch (a.ew) {
        case 0: return launch_step_gve<T, G, VEC, 0, PRIMAL>(a, s);
        case 16: return launch_step_gve<T, G, VEC, 16, PRIMAL>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int VEC, bool PRIMAL>
hipError_t launch_step_v(const StepArgs<T>& a, int lanes, hipStream_t s) {
    switch (lanes) {
        case 1: return launch_step_gv<T, 1, VEC, PRIMAL>(a, s);
        case 2: return launch_step_gv<T, 2, VEC, PRIMAL>(a, s);
        case 4: return launch_step_gv<T, 4, VEC, PRIMAL>(a, s);
        case 8: return launch_step_gv<T, 8, VEC, PRIMAL>(a, s);
        case 16: return launch_step_gv<T, 16, VEC, PRIMAL>(a, s);
        case 32: return launch_step_gv<T, 32, VEC, PRIMAL>(a, s);
        case 64: return launch_step_gv<T, 64, VEC, PRIMAL>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, bool PRIMAL>
hipError_t launch_step(const StepArgs<T>& a, int lanes, int vec, hipStream_t s) {
    if (a.wpb < 1 || a.wpb > 4) return hipErrorInvalidValue;
    if (a.ld % vec != 0) return hipErrorInvalidValue;
    switch (vec) {
        case 1: return launch_step_v<T, 1, PRIMAL>(a, lanes, s);
        case 2: return launch_step_v<T, 2, PRIMAL>(a, lanes, s);
        case 4: return launch_step_v<T, 4, PRIMAL>(a, lanes, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename T>
hipError_t launch_primal(const StepArgs<T>& a, int lanes, int vec, hipStream_t s) {
    return launch_step<T, true>(a, lanes, vec, s);
}
template <typename T>
hipError_t launch_dual(const StepArgs<T>& a, int lanes, int vec, hipStream_t s) {
    return launch_step<T, false>(a, lanes, vec, s);
}

// batches this narrow use k_eval_narrow (rows across the lanes)
constexpr int32_t EVAL_NARROW_COLS = 16;

template <typename T>
hipError_t launch_eval(const EvalArgs<T>& a, hipStream_t s) {
    if (a.ncols <= EVAL_NARROW_COLS) {
        const int64_t groups = ((int64_t)a.npx + a.npy + 7) / 8 * 8 * a.ncols;
        if (groups <= 0) return hipSuccess;
        if (a.kkt_only)
            hipLaunchKernelGGL((k_eval_narrow<T, true>), dim3((uint32_t)groups), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_eval_narrow<T, false>), dim3((uint32_t)groups), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const dim3 grid(a.npx + a.npy, (a.ncols + 63) / 64);
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
    if (a.kkt_only) hipLaunchKernelGGL((k_eval<T, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_eval<T, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tail(const TailArgs<T>& a, size_t dyn_lds, hipStream_t s) {
    if (a.ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tail<T>, dim3(a.ncols), dim3(TAIL_THREADS), dyn_lds, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce(const ControlArgs& a, hipStream_t s) {
    const int64_t pairs = (int64_t)2 * NTERM * a.ncols;
    if (pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3((uint32_t)((pairs + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_control(const ControlArgs& a, hipStream_t s) {
    if (a.batch_avg && a.ncols > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_control, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_compact(int32_t n, int32_t m, int32_t ld, int32_t ncols, T* const* blk,
                          T* const* res, const RetireEntry* retire, const MoveEntry* moves,
                          const int32_t* fresh, Slots sl, Globals* g, hipStream_t s) {
    constexpr int TR = 256 / (int)sizeof(T);
    Blocks8<T> B{}, R{};
    for (int b = 0; b < 8; ++b) B.b[b] = blk[b];
    for (int b = 0; b < 4; ++b) R.b[b] = res[b];
    const int64_t tiles = ((int64_t)n + TR - 1) / TR + ((int64_t)m + TR - 1) / TR;
    (void)ncols;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((uint32_t)(tiles > 0 ? tiles : 1));
    hipLaunchKernelGGL(k_compact<T>, grid, dim3(256), 0, s, n, m, ld, B, R, retire, moves, fresh,
                       sl, g);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_blocks(int32_t n, int32_t m, int32_t ld, int32_t ncols, Slots sl,
                              const double* xl, const double* xu, const double* xw,
                              const double* yw, int32_t mode, T* Xbar, T* X0, T* Y, T* Y0,
                              hipStream_t s) {
    const int64_t total = (int64_t)(n + m) * ld;
    if (total == 0) return hipSuccess;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_init_blocks<T>, dim3((uint32_t)blocks), dim3(256), 0, s, n, m, ld, ncols,
                       sl, xl, xu, xw, yw, mode, Xbar, X0, Y, Y0);
    return hipGetLastError();
}

hipError_t launch_begin_solve(Slots sl, SlotCtl* ctl, int32_t ncols, int32_t max_iters, Globals* g,
                              double tol, hipStream_t s) {
    const int32_t blocks = (ncols + 255) / 256;
    hipLaunchKernelGGL(k_begin_solve, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, sl, ctl,
                       ncols, max_iters, g, tol);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_columns(int32_t n, int32_t m, int32_t ld, int32_t c0, int32_t cnt, Slots sl,
                               const double* xl, const double* xu, const double* xw,
                               const double* yw, int32_t mode, T* const* blk, hipStream_t s) {
    Blocks8<T> B{};
    for (int b = 0; b < 8; ++b) B.b[b] = blk[b];
    const int64_t total = ((int64_t)n + m) * cnt;
    if (total == 0) return hipSuccess;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_init_columns<T>, dim3((uint32_t)blocks), dim3(256), 0, s, n, m, ld, c0, cnt,
                       sl, xl, xu, xw, yw, mode, B);
    return hipGetLastError();
}

hipError_t launch_admit(SlotCtl* ctl, const int32_t* rows, const SlotCtl* src, int32_t cnt,
                        Globals* g, int32_t n_cols, hipStream_t s) {
    const int32_t blocks = (cnt + 255) / 256;
    hipLaunchKernelGGL(k_admit, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, ctl, rows, src, cnt,
                       g, n_cols);
    return hipGetLastError();
}

hipError_t launch_rescale(double* v, const double* d, int64_t count, int32_t period,
                          int32_t divide, hipStream_t s) {
    if (count == 0 || period == 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rescale, dim3((uint32_t)blocks), dim3(256), 0, s, v, d, count, period,
                       divide);
    return hipGetLastError();
}

hipError_t launch_widen(const float* src, int64_t count, double* dst, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_widen, dim3((uint32_t)blocks), dim3(256), 0, s, src, count, dst);
    return hipGetLastError();
}

hipError_t launch_spmv(const int32_t* rp, const int32_t* ci, const double* v, int32_t rows,
                       const double* x, double* y, hipStream_t s) {
    if (rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spmv, dim3((rows + 255) / 256), dim3(256), 0, s, rp, ci, v, rows, x, y);
    return hipGetLastError();
}

hipError_t launch_norm2sq(const double* x, int32_t len, double* partial, double* out,
                          hipStream_t s) {
    int32_t blocks = (len + 255) / 256;
    if (blocks > NORM_BLOCKS) blocks = NORM_BLOCKS;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_norm_partial, dim3(blocks), dim3(256), 0, s, x, len, partial);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, partial, blocks, out);
    return hipGetLastError();
}

hipError_t launch_scale(double* x, int32_t len, const double* nrm2sq, hipStream_t s) {
    if (len == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale, dim3((len + 255) / 256), dim3(256), 0, s, x, len, nrm2sq);
    return hipGetLastError();
}

hipError_t launch_fill(double* x, int32_t len, double v, hipStream_t s) {
    if (len == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((len + 255) / 256), dim3(256), 0, s, x, len, v);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sp_iterate(const SharedArgs<T>& a, hipStream_t s) {
    if (a.n > 0) hipLaunchKernelGGL(k_sp_primal<T>, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    if (a.m > 0) hipLaunchKernelGGL(k_sp_dual<T>, dim3((a.m + 255) / 256), dim3(256), 0, s, a);
    if (a.nslots > 0)
        hipLaunchKernelGGL(k_sp_side<T>, dim3((a.nslots + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sp_eval(const SharedArgs<T>& a, hipStream_t s) {
    const int32_t np = a.npx + a.npy;
    if (np == 0 || a.nslots == 0) return hipSuccess;
    if (a.npx > 2048 || a.npy > 2048 || a.ncls < 1 || a.ncls > 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sp_terms<T>, dim3(np, a.ncls), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sp_bcast<T>, dim3(np, (a.nslots + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sp_touched<T>, dim3(a.nslots, SP_SPLIT), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sp_place(const SharedArgs<T>& a, hipStream_t s) {
    if (a.nslots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sp_map<T>, dim3(1), dim3(1024), 0, s, a);
    const int64_t total = (int64_t)a.n + a.m;
    const uint32_t gd = (uint32_t)(total < 16384 ? total : 16384);
    hipLaunchKernelGGL(k_sp_dense<T>, dim3(gd), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sp_results<T>, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sp_patch<T>, dim3((2 * a.nslots + 3) / 4), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sp_finish, dim3(1), dim3(1024), 0, s, a.sl, a.moves, a.g);
    return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_sp_iterate<double>(const SharedArgs<double>&, hipStream_t);
template hipError_t launch_sp_iterate<float>(const SharedArgs<float>&, hipStream_t);
template hipError_t launch_sp_eval<double>(const SharedArgs<double>&, hipStream_t);
template hipError_t launch_sp_eval<float>(const SharedArgs<float>&, hipStream_t);
template hipError_t launch_sp_place<double>(const SharedArgs<double>&, hipStream_t);
template hipError_t launch_sp_place<float>(const SharedArgs<float>&, hipStream_t);
template hipError_t launch_primal<double>(const StepArgs<double>&, int, int, hipStream_t);
template hipError_t launch_primal<float>(const StepArgs<float>&, int, int, hipStream_t);
template hipError_t launch_dual<double>(const StepArgs<double>&, int, int, hipStream_t);
template hipError_t launch_dual<float>(const StepArgs<float>&, int, int, hipStream_t);
template hipError_t launch_tail<double>(const TailArgs<double>&, size_t, hipStream_t);
template hipError_t launch_tail<float>(const TailArgs<float>&, size_t, hipStream_t);
template hipError_t launch_eval<double>(const EvalArgs<double>&, hipStream_t);
template hipError_t launch_eval<float>(const EvalArgs<float>&, hipStream_t);
template hipError_t launch_compact<double>(int32_t, int32_t, int32_t, int32_t, double* const*,
                                           double* const*, const RetireEntry*, const MoveEntry*,
                                           const int32_t*, Slots, Globals*, hipStream_t);
template hipError_t launch_compact<float>(int32_t, int32_t, int32_t, int32_t, float* const*,
                                          float* const*, const RetireEntry*, const MoveEntry*,
                                          const int32_t*, Slots, Globals*, hipStream_t);
template hipError_t launch_init_columns<double>(int32_t, int32_t, int32_t, int32_t, int32_t, Slots,
                                                const double*, const double*, const double*,
                                                const double*, int32_t, double* const*,
                                                hipStream_t);
template hipError_t launch_init_columns<float>(int32_t, int32_t, int32_t, int32_t, int32_t, Slots,
                                               const double*, const double*, const double*,
                                               const double*, int32_t, float* const*, hipStream_t);
template hipError_t launch_init_blocks<double>(int32_t, int32_t, int32_t, int32_t, Slots,
                                               const double*, const double*, const double*,
                                               const double*, int32_t, double*, double*, double*,
                                               double*, hipStream_t);
template hipError_t launch_init_blocks<float>(int32_t, int32_t, int32_t, int32_t, Slots,
                                              const double*, const double*, const double*,
                                              const double*, int32_t, float*, float*, float*,
                                              float*, hipStream_t);

}  // namespace pdlpb
