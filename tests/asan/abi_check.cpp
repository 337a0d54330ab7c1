// C ABI test program for host-side AddressSanitizer builds.  Without arguments: input
// validation of pdlpb_create, every entry point with a NULL context, and (when
// no device is present) the device-failure path.  With --device: one context
// through solve, getters, bound tightening, branching scores, device-pointer
// inputs, a serving session, and the other precision, restart scope and
// scaling options.  Exit status 0 when every check holds.
#include "pdlpb.h"
#include <hip/hip_runtime_api.h>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

static int n_fail = 0;
#define EXPECT(cond) do { if (!(cond)) { printf("FAIL line %d: %s\n", __LINE__, #cond); ++n_fail; } } while (0)

struct LP {
    int32_t m = 2, n = 3;
    std::vector<int64_t> rp{0, 2, 3};
    std::vector<int32_t> ci{0, 2, 1};
    std::vector<double> val{1.0, 2.0, -1.0}, c{1.0, 0.5, -1.0}, b{1.0, 2.0}, l{0, 0, 0}, u{4, 4, 4};
    std::vector<char> sense{'E', 'L'};
    int create(pdlpb_ctx** out, const pdlpb_options* o = nullptr) {
        return pdlpb_create(out, m, n, (int64_t)ci.size(), rp.data(), ci.data(), val.data(), c.data(),
                            b.data(), sense.data(), l.data(), u.data(), o);
    }
};


// A feasible random LP: m rows (half E, half L), n columns with 4 nonzeros each, box [0, 10].
static void make_lp(int m, int n, uint64_t seed, std::vector<int64_t>& rp, std::vector<int32_t>& ci,
                    std::vector<double>& val, std::vector<double>& c, std::vector<double>& b,
                    std::vector<char>& sense, std::vector<double>& l, std::vector<double>& u) {
    uint64_t st = seed;
    auto rnd = [&]() { st = st * 6364136223846793005ULL + 1442695040888963407ULL; return (double)(st >> 11) / 9007199254740992.0; };
    std::vector<std::vector<std::pair<int32_t, double>>> rows(m);
    for (int j = 0; j < n; ++j) {
        int picked[4]; int np = 0;
        while (np < 4) {
            int r = (int)(rnd() * m); bool dup = false;
            for (int q = 0; q < np; ++q) dup |= picked[q] == r;
            if (!dup) picked[np++] = r;
        }
        for (int q = 0; q < 4; ++q) rows[picked[q]].push_back({j, 2.0 * rnd() - 1.0});
    }
    std::vector<double> x0(n);
    for (int j = 0; j < n; ++j) x0[j] = 10.0 * rnd();
    rp.assign(1, 0); ci.clear(); val.clear(); b.assign(m, 0.0); sense.assign(m, 'E');
    for (int i = 0; i < m; ++i) {
        for (auto& e : rows[i]) { ci.push_back(e.first); val.push_back(e.second); b[i] += e.second * x0[e.first]; }
        rp.push_back((int64_t)ci.size());
        if (i >= m / 2) { sense[i] = 'L'; b[i] += 1.0; }
    }
    c.resize(n);
    for (int j = 0; j < n; ++j) c[j] = 2.0 * rnd() - 1.0;
    l.assign(n, 0.0); u.assign(n, 10.0);
}

static int device_section() {
    const int m = 40, n = 100;
    std::vector<int64_t> rp; std::vector<int32_t> ci; std::vector<double> val, c, b, l, u; std::vector<char> sense;
    make_lp(m, n, 12345, rp, ci, val, c, b, sense, l, u);
    pdlpb_ctx* x = nullptr;
    int rc = pdlpb_create(&x, m, n, (int64_t)ci.size(), rp.data(), ci.data(), val.data(), c.data(), b.data(),
                          sense.data(), l.data(), u.data(), nullptr);
    if (rc < 0) { printf("create: %d %s\n", rc, pdlpb_last_error(nullptr)); return 1; }
    const int B = 10;
    pdlpb_delta d[B] = {{PDLPB_BASE, 0, 0.0}, {PDLPB_SET_LO, 3, 5.0}, {PDLPB_SET_HI, 3, 2.0},
                        {PDLPB_SET_LO, 7, 11.0}, {PDLPB_OBJ_UNIT, 5, 1.0}, {PDLPB_OBJ_UNIT, 5, -1.0},
                        {PDLPB_SET_HI, 9, NAN}, {PDLPB_BASE, 0, 0.0}, {PDLPB_OBJ_UNIT, 50, 1.0},
                        {PDLPB_OBJ_UNIT, 50, -1.0}};
    EXPECT(pdlpb_set_batch(x, B, d, nullptr, nullptr, nullptr, PDLPB_WARM_NONE, PDLPB_MEM_HOST) == 0);
    EXPECT(pdlpb_solve(x, 1e-6, 50000) == 0);
    std::vector<double> X((size_t)B * n), Y((size_t)B * m), kkt(4 * B), obj(B), xs(n), ys(m), xi(n), yi(m);
    std::vector<int32_t> st(B); std::vector<int64_t> it(B);
    EXPECT(pdlpb_get_batch(x, X.data(), Y.data(), st.data(), kkt.data(), obj.data(), it.data(), PDLPB_MEM_HOST) == 0);
    for (int j = 0; j < B; ++j) {
        int32_t s1, nr, lg[8]; double k4[4], o1, w; int64_t i1;
        EXPECT(pdlpb_get(x, j, xs.data(), ys.data(), &s1, k4, &o1, &i1, PDLPB_MEM_HOST) == 0);
        EXPECT(s1 == st[j] && i1 == it[j] && std::memcmp(xs.data(), &X[(size_t)j * n], n * 8) == 0);
        EXPECT(pdlpb_get_trace(x, j, xi.data(), yi.data(), &w, &nr, lg, 8) == 0);
        printf("LP %d: status %d iters %lld obj %.6f restarts %d\n", j, s1, (long long)i1, o1, nr);
    }
    EXPECT(st[0] == PDLPB_STATUS_OPTIMAL && st[6] != PDLPB_STATUS_OPTIMAL && st[3] != PDLPB_STATUS_OPTIMAL);
    int32_t s1; double k4[4], o1; int64_t i1;
    EXPECT(pdlpb_get(x, B, nullptr, nullptr, &s1, k4, &o1, &i1, PDLPB_MEM_HOST) < 0);
    EXPECT(pdlpb_get(x, -1, nullptr, nullptr, &s1, k4, &o1, &i1, PDLPB_MEM_HOST) < 0);
    std::vector<double> dobj(B), lo(n), hi(n), gain(B), score(B), dr(m), dc(n);
    EXPECT(pdlpb_get_dual_objective(x, dobj.data()) == 0);
    int32_t nc = -1, inf = -1;
    EXPECT(pdlpb_obbt_tighten(x, 1e-8, 1e-4, lo.data(), hi.data(), &nc, &inf) == 0);
    EXPECT(pdlpb_branch_scores(x, obj[0], 1.0 / 6, gain.data(), score.data()) == 0);
    EXPECT(pdlpb_get_scaling(x, dr.data(), dc.data()) == 0);
    double eta, na;
    EXPECT(pdlpb_get_step_size(x, &eta, &na) == 0 && eta > 0 && na > 0);
    EXPECT(pdlpb_device_bytes(x) > 0);
    EXPECT(pdlpb_set_kernel_timing(x, 1) == 0);
    EXPECT(pdlpb_set_batch(x, B, d, nullptr, nullptr, nullptr, PDLPB_WARM_NONE, PDLPB_MEM_HOST) == 0);
    EXPECT(pdlpb_solve(x, 1e-6, 50000) == 0);
    int64_t cnt[4], cols[4]; double tms[4];
    EXPECT(pdlpb_kernel_times(x, cnt, tms) == 0 && cnt[0] > 0);
    EXPECT(pdlpb_kernel_columns(x, cols) == 0);
    EXPECT(pdlpb_set_kernel_timing(x, 0) == 0);
    // another tile shape sums every row in the same order: identical results
    EXPECT(pdlpb_set_tile(x, 4, 2) == 0);
    EXPECT(pdlpb_set_batch(x, B, d, nullptr, nullptr, nullptr, PDLPB_WARM_NONE, PDLPB_MEM_HOST) == 0);
    EXPECT(pdlpb_solve(x, 1e-6, 50000) == 0);
    std::vector<double> obj2(B); std::vector<int64_t> it2(B);
    EXPECT(pdlpb_get_batch(x, nullptr, nullptr, nullptr, nullptr, obj2.data(), it2.data(), PDLPB_MEM_HOST) == 0);
    for (int j = 0; j < B; ++j) EXPECT(it2[j] == it[j] && (obj2[j] == obj[j] || (std::isnan(obj2[j]) && std::isnan(obj[j]))));
    EXPECT(pdlpb_set_tile(x, 0, 0) == 0);
    // device pointers: deltas, per-LP warm starts and results in device memory
    {
        pdlpb_delta* dd = nullptr; double *dx = nullptr, *dy = nullptr, *dw = nullptr, *dX = nullptr;
        EXPECT(hipMalloc(&dd, sizeof(d)) == hipSuccess && hipMalloc(&dx, X.size() * 8) == hipSuccess &&
               hipMalloc(&dy, Y.size() * 8) == hipSuccess && hipMalloc(&dw, B * 8) == hipSuccess &&
               hipMalloc(&dX, X.size() * 8) == hipSuccess);
        std::vector<double> w(B, 1.0);
        EXPECT(hipMemcpy(dd, d, sizeof(d), hipMemcpyHostToDevice) == hipSuccess);
        EXPECT(hipMemcpy(dx, X.data(), X.size() * 8, hipMemcpyHostToDevice) == hipSuccess);
        EXPECT(hipMemcpy(dy, Y.data(), Y.size() * 8, hipMemcpyHostToDevice) == hipSuccess);
        EXPECT(hipMemcpy(dw, w.data(), B * 8, hipMemcpyHostToDevice) == hipSuccess);
        EXPECT(pdlpb_set_batch(x, B, dd, dx, dy, dw, PDLPB_WARM_PER_LP, PDLPB_MEM_DEVICE) == 0);
        EXPECT(pdlpb_solve(x, 1e-6, 50000) == 0);
        EXPECT(pdlpb_get_batch(x, dX, nullptr, st.data(), nullptr, nullptr, nullptr, PDLPB_MEM_DEVICE) == 0);
        EXPECT(st[0] == PDLPB_STATUS_OPTIMAL);
        (void)hipFree(dd); (void)hipFree(dx); (void)hipFree(dy); (void)hipFree(dw); (void)hipFree(dX);
    }
    // serving: base warm start, admission control, poll / result / release
    EXPECT(pdlpb_set_base_warm(x, &X[0], &Y[0], 1.0, PDLPB_MEM_HOST) == 0);
    EXPECT(pdlpb_serve_begin(x, 8) == 0);
    int64_t first = -1;
    EXPECT(pdlpb_submit(x, 6, d, PDLPB_WARM_BASE, 1e-6, 50000, PDLPB_MEM_HOST, &first) == 0);
    int64_t first2 = -1;
    EXPECT(pdlpb_submit(x, 4, d + 6, PDLPB_WARM_NONE, 1e-6, 50000, PDLPB_MEM_HOST, &first2) == PDLPB_ENOMEM);
    int got = 0, submitted = 6, rounds = 0;
    bool more = false;
    while (got < submitted && rounds < 200000) {
        ++rounds;
        int32_t run, q, k;
        EXPECT(pdlpb_serve_launch(x) == 0);
        EXPECT(pdlpb_serve_wait(x, &run, &q) == 0);
        int64_t ids[16];
        EXPECT(pdlpb_poll(x, ids, 16, &k) == 0);
        for (int i = 0; i < k; ++i) {
            EXPECT(pdlpb_result(x, ids[i], xs.data(), ys.data(), &s1, k4, &o1, &i1, PDLPB_MEM_HOST) == 0);
            EXPECT(pdlpb_release(x, ids[i]) == 0);
            EXPECT(pdlpb_release(x, ids[i]) < 0);
            EXPECT(pdlpb_result(x, ids[i], nullptr, nullptr, &s1, k4, &o1, &i1, PDLPB_MEM_HOST) < 0);
            ++got;
        }
        if (!more && got >= 2) {
            EXPECT(pdlpb_submit(x, 4, d + 6, PDLPB_WARM_NONE, 1e-6, 50000, PDLPB_MEM_HOST, &first2) == 0);
            submitted += 4;
            more = true;
        }
    }
    printf("served %d LPs in %d rounds\n", got, rounds);
    EXPECT(got == submitted);
    EXPECT(pdlpb_serve_begin(x, 4) == 0);
    pdlpb_destroy(x);
    // the other precision, the batch-average scope and problem scaling
    for (int variant = 0; variant < 3; ++variant) {
        pdlpb_options o; pdlpb_default_options(&o);
        if (variant == 0) o.precision = PDLPB_MIXED32;
        if (variant == 1) o.restart_scope = PDLPB_RESTART_BATCH_AVG;
        if (variant == 2) o.scaling = 1;
        x = nullptr;
        EXPECT(pdlpb_create(&x, m, n, (int64_t)ci.size(), rp.data(), ci.data(), val.data(), c.data(), b.data(),
                            sense.data(), l.data(), u.data(), &o) == 0);
        if (!x) continue;
        EXPECT(pdlpb_set_batch(x, 6, d, nullptr, nullptr, nullptr, PDLPB_WARM_NONE, PDLPB_MEM_HOST) == 0);
        EXPECT(pdlpb_solve(x, 1e-4, 50000) == 0);
        EXPECT(pdlpb_get_batch(x, X.data(), Y.data(), st.data(), kkt.data(), obj.data(), it.data(), PDLPB_MEM_HOST) == 0);
        printf("variant %d: LP 0 status %d iters %lld obj %.6f\n", variant, st[0], (long long)it[0], obj[0]);
        EXPECT(st[0] == PDLPB_STATUS_OPTIMAL);
        pdlpb_destroy(x);
    }
    return 0;
}

int main(int argc, char** argv) {
    pdlpb_ctx* x = reinterpret_cast<pdlpb_ctx*>(0x1);
    // malformed input, each rejected before any device call
    { LP p; p.rp[0] = 1; EXPECT(p.create(&x) < 0 && x == nullptr); }
    { LP p; p.rp = {0, 3, 2}; EXPECT(p.create(&x) < 0); }
    { LP p; p.rp = {0, 2, 5}; EXPECT(p.create(&x) < 0); }
    { LP p; p.rp = {0, 2, (int64_t)1 << 40}; EXPECT(p.create(&x) < 0); }
    { LP p; p.ci = {2, 0, 1}; EXPECT(p.create(&x) < 0); }
    { LP p; p.ci = {0, 3, 1}; EXPECT(p.create(&x) < 0); }
    { LP p; p.ci = {0, -1, 1}; EXPECT(p.create(&x) < 0); }
    { LP p; p.val[1] = NAN; EXPECT(p.create(&x) < 0); }
    { LP p; p.c[0] = INFINITY; EXPECT(p.create(&x) < 0); }
    { LP p; p.b[1] = NAN; EXPECT(p.create(&x) < 0); }
    { LP p; p.sense[1] = 'Q'; EXPECT(p.create(&x) < 0); }
    { LP p; p.l[0] = INFINITY; EXPECT(p.create(&x) < 0); }
    { LP p; p.u[0] = -INFINITY; EXPECT(p.create(&x) < 0); }
    { LP p; p.l[2] = 5.0; EXPECT(p.create(&x) < 0); }
    { LP p; p.u[1] = NAN; EXPECT(p.create(&x) < 0); }
    { LP p; p.m = -1; EXPECT(p.create(&x) < 0); }
    { LP p; p.n = 0; EXPECT(p.create(&x) < 0); }
    { LP p; EXPECT(pdlpb_create(&x, p.m, p.n, 3, p.rp.data(), nullptr, p.val.data(), p.c.data(),
                                p.b.data(), p.sense.data(), p.l.data(), p.u.data(), nullptr) < 0); }
    { LP p; EXPECT(pdlpb_create(nullptr, p.m, p.n, 3, p.rp.data(), p.ci.data(), p.val.data(), p.c.data(),
                                p.b.data(), p.sense.data(), p.l.data(), p.u.data(), nullptr) < 0); }
    // bad options
    {
        LP p; pdlpb_options o;
        pdlpb_default_options(&o); o.struct_size -= 8; EXPECT(p.create(&x, &o) < 0);
        pdlpb_default_options(&o); o.eval_every = 1; EXPECT(p.create(&x, &o) < 0);
        pdlpb_default_options(&o); o.theta = 2.0; EXPECT(p.create(&x, &o) < 0);
        pdlpb_default_options(&o); o.step_size = NAN; EXPECT(p.create(&x, &o) < 0);
        pdlpb_default_options(&o); o.cross_sign = 0.5; EXPECT(p.create(&x, &o) < 0);
        pdlpb_default_options(&o); o.max_batch = 5000; EXPECT(p.create(&x, &o) < 0);
        pdlpb_default_options(&o); o.tile_lanes = 3; EXPECT(p.create(&x, &o) < 0);
        pdlpb_default_options(&o); o.tile_vec = 3; EXPECT(p.create(&x, &o) < 0);
        pdlpb_default_options(&o); o.precision = 7; EXPECT(p.create(&x, &o) < 0);
    }
    const char* msg = pdlpb_last_error(nullptr);
    EXPECT(msg && std::strlen(msg) > 0);
    printf("last create error: %s\n", msg);
    // well-formed input without a device: a clean device error, nothing left allocated
    const bool on_device = argc > 1 && std::strcmp(argv[1], "--device") == 0;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess) n_dev = 0;
    for (int prec = 0; prec < 2 && n_dev == 0; ++prec) {
        LP p; pdlpb_options o; pdlpb_default_options(&o); o.precision = prec;
        int rc = p.create(&x, &o);
        printf("create without a device: rc=%d (%s)\n", rc, pdlpb_last_error(nullptr));
        EXPECT(rc < 0 && x == nullptr);
    }
    // every entry point rejects a NULL context
    double d4[4], d; int32_t i32, i32b; int64_t i64, i64a[4]; double dd[4];
    pdlpb_delta del{0, 0, 0.0};
    EXPECT(pdlpb_set_batch(nullptr, 1, &del, nullptr, nullptr, nullptr, 0, 0) < 0);
    EXPECT(pdlpb_solve(nullptr, 1e-4, 10) < 0);
    EXPECT(pdlpb_get(nullptr, 0, nullptr, nullptr, &i32, d4, &d, &i64, 0) < 0);
    EXPECT(pdlpb_get_batch(nullptr, nullptr, nullptr, &i32, d4, &d, &i64, 0) < 0);
    EXPECT(pdlpb_get_trace(nullptr, 0, nullptr, nullptr, &d, &i32, &i32b, 1) < 0);
    EXPECT(pdlpb_get_dual_objective(nullptr, &d) < 0);
    EXPECT(pdlpb_obbt_tighten(nullptr, 1e-6, 0.0, &d, &d, &i32, &i32b) < 0);
    EXPECT(pdlpb_branch_scores(nullptr, 0.0, 1.0 / 6, &d, &d) < 0);
    EXPECT(pdlpb_set_base_warm(nullptr, &d, &d, 1.0, 0) < 0);
    EXPECT(pdlpb_serve_begin(nullptr, 4) < 0);
    EXPECT(pdlpb_submit(nullptr, 1, &del, 0, 1e-4, 10, 0, &i64) < 0);
    EXPECT(pdlpb_serve_launch(nullptr) < 0);
    EXPECT(pdlpb_serve_wait(nullptr, &i32, &i32b) < 0);
    EXPECT(pdlpb_poll(nullptr, &i64, 1, &i32) < 0);
    EXPECT(pdlpb_result(nullptr, 0, nullptr, nullptr, &i32, d4, &d, &i64, 0) < 0);
    EXPECT(pdlpb_release(nullptr, 0) < 0);
    EXPECT(pdlpb_set_tile(nullptr, 1, 1) < 0);
    EXPECT(pdlpb_get_scaling(nullptr, &d, &d) < 0);
    EXPECT(pdlpb_get_step_size(nullptr, &d, &d) < 0);
    EXPECT(pdlpb_set_kernel_timing(nullptr, 1) < 0);
    EXPECT(pdlpb_kernel_times(nullptr, i64a, dd) < 0);
    EXPECT(pdlpb_kernel_columns(nullptr, i64a) < 0);
    EXPECT(pdlpb_device_bytes(nullptr) <= 0);
    pdlpb_destroy(nullptr);
    if (on_device) EXPECT(device_section() == 0);
    printf("%s (%d failures)\n", n_fail ? "FAILED" : "ok", n_fail);
    return n_fail ? 1 : 0;
}
