// Host-only check of the library's runtime (validation, the chunked launch
// schedule of rd_step, output-buffer binding, the stop-decision state machine,
// serving admission / batching / retirement, the adaptive step rule, context
// teardown), built as plain C++ against the HIP stub in tests/hoststub and run
// under AddressSanitizer + UndefinedBehaviorSanitizer by tests/test_host_sanitized.py.
//
// The kernels are replaced by a scripted "device" whose launches follow the
// control flow of the real ones (which launch skips, which buffer an iteration
// reads and writes, who takes the stop decision) and whose stop decisions call
// the same decide() the kernels call.  Its residual model: after n iterations of
// an FP64 step, ||F/h_t|| = q^n with q = h_t / (h_t + 0.01) (q = 3, divergence, for
// h_t >= 1), and every iteration adds 1 to the iterate, so a step's result is
// u_n + iterations; the mixed path's inner loop runs on a correction that counts
// its iterations, its outer update adds it to U, and the inner norm after j inner
// iterations is (outer norm) q^j.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../include/rd.h"
#include "../paper_2305_03945_amd/csrc/registry.h"

using namespace rdk;

static int g_fail = 0;
#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++g_fail;                                                                 \
        }                                                                             \
    } while (0)

namespace rdk {
KSet g_kernels[2][LOGN_MAX + 1][2][EQ_COUNT];
KSet g_kernels3[2][LOGN3_MAX + 1][2][EQ_COUNT];
}  // namespace rdk

namespace {

double model_q(double ht) { return ht >= 1.0 ? 3.0 : ht / (ht + 0.01); }
size_t npts(const Slot &s) { return (size_t)s.N * s.N; }

bool skip(int kind, const State &st) {
    if (kind == K_INIT64 || kind == K_OUTER_INIT) return false;
    if (kind == K_OUTER_UPD) return st.outer_done || !st.done;
    if (kind == K_MIXED) return st.outer_done != 0;
    return st.done != 0;
}

// Partial sums of a residual pass with norm res: block 0 carries everything.
void write_partials(Slot &s, double res, double mass) {
    const int C = s.ncomp;
    std::memset(s.partials, 0, (size_t)s.nblk_rows * 2 * C * sizeof(double));
    for (int c = 0; c < C; ++c) {
        const double w = res * s.ht / C;
        s.partials[c] = w * w;
        s.partials[C + c] = c == 0 ? mass : 0.0;
    }
}

template <int KIND> void decide_from_partials(Slot &s) {
    const int C = s.ncomp;
    double res = 0.0, m = 0.0;
    for (int c = 0; c < C; ++c) {
        double sq = 0.0, mm = 0.0;
        for (int b = 0; b < s.nblk_rows; ++b) {
            sq += s.partials[b * 2 * C + c];
            mm += s.partials[b * 2 * C + C + c];
        }
        res += std::sqrt(sq);
        m += mm;
    }
    res /= s.ht;
    const StopRule rule{s.tol, s.inner_rtol, s.max_iter, s.max_outer};
    *s.st = decide<KIND>(*s.st, rule, res, m);
}

double field_mass(const double *U, const double *Uk, size_t n) {
    double m = 0.0;
    for (size_t i = 0; i < n; ++i) m += U[i] - Uk[i];
    return m;
}

// FP64 residual of iterate U: q^(U - U^k) (the iterate counts its iterations).
double res64(const Slot &s, const double *U) {
    const double n = U[0] - s.Uk[0];
    return std::pow(model_q(s.ht), n);
}

template <int MODE, int KIND0> void f_init(Slot *const *slots, int nslots, hipStream_t, hipEvent_t *) {
    for (int i = 0; i < nslots; ++i) {
        Slot &s = *slots[i];
        const size_t n = (size_t)s.ncomp * npts(s);
        std::memcpy(s.Uk, s.src, n * sizeof(double));
        double *U = MODE == MODE_F64 ? (double *)s.U[0] : s.U64[0];
        std::memcpy(U, s.src, n * sizeof(double));
        if (MODE == MODE_MIXED)
            for (size_t j = 0; j < n; ++j) {
                s.r32[j] = 0.f;
                s.Ub32[j] = (float)U[j];
            }
        write_partials(s, res64(s, U), 0.0);
        decide_from_partials<KIND0>(s);
    }
}

template <int FIN> void f_cols(Slot *const *slots, int nslots, hipStream_t, hipEvent_t *) {
    for (int i = 0; i < nslots; ++i) {
        Slot &s = *slots[i];
        if (FIN >= 0 && !skip(FIN, *s.st)) decide_from_partials<FIN>(s);
    }
}

void f_rowinv(Slot *const *, int, hipStream_t, hipEvent_t *) {}

template <int MODE> void f_upd(Slot *const *slots, int nslots, hipStream_t, hipEvent_t *) {
    for (int i = 0; i < nslots; ++i) {
        Slot &s = *slots[i];
        if (s.st->done) continue;
        const int it = s.st->iters;
        const size_t n = (size_t)s.ncomp * npts(s);
        if (MODE == MODE_F64) {
            const double *a = (const double *)s.U[it & 1];
            double *b = (double *)s.U[(it + 1) & 1];
            for (size_t j = 0; j < n; ++j) b[j] = a[j] + 1.0;
        } else {
            const float *a = (const float *)s.U[it & 1];
            float *b = (float *)s.U[(it + 1) & 1];
            for (size_t j = 0; j < n; ++j) b[j] = (it == 0 ? 0.f : a[j]) + 1.f;
        }
    }
}

template <int MODE> void f_rowfwd(Slot *const *slots, int nslots, hipStream_t, hipEvent_t *) {
    for (int i = 0; i < nslots; ++i) {
        Slot &s = *slots[i];
        const State st = *s.st;
        const size_t n = (size_t)s.ncomp * npts(s);
        if (MODE == MODE_F64) {
            if (skip(K_ITER64, st)) continue;
            const double *U = (const double *)s.U[(st.iters + 1) & 1];
            write_partials(s, res64(s, U), field_mass(U, s.Uk, n));
        } else if (!skip(K_MIXED, st)) {
            if (st.done) {
                // outer update U += e
                const double *a = s.U64[st.outer & 1];
                double *b = s.U64[(st.outer + 1) & 1];
                const float *e = (const float *)s.U[st.iters & 1];
                for (size_t j = 0; j < n; ++j) b[j] = a[j] + (st.iters > 0 ? (double)e[j] : 0.0);
                write_partials(s, res64(s, b), field_mass(b, s.Uk, n));
            } else {
                const float *e = (const float *)s.U[(st.iters + 1) & 1];
                write_partials(s, st.outer_res * std::pow(model_q(s.ht), (double)e[0]), 0.0);
            }
        }
    }
}

template <int KIND> void f_fin(Slot *const *slots, int nslots, hipStream_t, hipEvent_t *) {
    for (int i = 0; i < nslots; ++i) {
        Slot &s = *slots[i];
        if (!skip(KIND, *s.st)) decide_from_partials<KIND>(s);
    }
}

// The whole step in one launch (the device's k_step_wg): the same launches in
// order until every slot has finished.
template <int MODE> void f_step_wg(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *) {
    constexpr int KIT = MODE == MODE_F64 ? K_ITER64 : K_MIXED;
    f_init<MODE, MODE == MODE_F64 ? K_INIT64 : K_OUTER_INIT>(slots, nslots, st, nullptr);
    for (int guard = 0; guard < 1000000; ++guard) {
        bool all = true;
        for (int i = 0; i < nslots; ++i) all = all && slots[i]->st->outer_done;
        if (all) break;
        f_upd<MODE>(slots, nslots, st, nullptr);
        f_rowfwd<MODE>(slots, nslots, st, nullptr);
        f_fin<KIT>(slots, nslots, st, nullptr);
    }
}

void f_tin(Slot *const *, int, const double *, double *, hipStream_t) {}
void f_tout(Slot *const *, int, const double *, double *, hipStream_t) {}

void fill(int L) {
    for (int mode = 0; mode < 2; ++mode)
        for (int bc = 0; bc < 2; ++bc)
            for (int eq = 0; eq < EQ_COUNT; ++eq) {
                if (mode == MODE_MIXED && eq == EQ_FCH) continue;   // FP64 only, as in the library
                KSet &k = g_kernels[mode][L][bc][eq];
                if (mode == MODE_F64) {
                    k.init = f_init<MODE_F64, K_INIT64>;
                    k.cols_fin = f_cols<K_ITER64>;
                    k.fin = f_fin<K_ITER64>;
                    k.upd = f_upd<MODE_F64>;
                    k.rowfwd = f_rowfwd<MODE_F64>;
                } else {
                    k.init = f_init<MODE_MIXED, K_OUTER_INIT>;
                    k.cols_fin = f_cols<K_MIXED>;
                    k.fin = f_fin<K_MIXED>;
                    k.upd = f_upd<MODE_MIXED>;
                    k.rowfwd = f_rowfwd<MODE_MIXED>;
                }
                k.cols = f_cols<-1>;
                k.rowinv = f_rowinv;
                k.tin = f_tin;
                k.tout = f_tout;
                k.rows_per_block = 2;
                k.dim = 2;
                // small grids (N <= 32 here) take the single-launch step
                if (L <= 5 && eq != EQ_FCH)
                    k.step_wg = mode == MODE_F64 ? f_step_wg<MODE_F64> : f_step_wg<MODE_MIXED>;
            }
}

}  // namespace

namespace rdk {
static unsigned char g_scratch_host[NOALLOC_BYTES];
hipError_t noalloc_scratch_address(void **out) {
    *out = g_scratch_host;
    return hipSuccess;
}
void register_upd_kernels() {}
#define RD_REG(L) \
    void register_logn_##L() { fill(L); }
RD_REG(4) RD_REG(5) RD_REG(6) RD_REG(7) RD_REG(8) RD_REG(9) RD_REG(10) RD_REG(11) RD_REG(12)
#undef RD_REG

void launch_residual(int, int, const Slot *, int N, const double *U, const double *Uk, double *W, double *partials,
                     hipStream_t) {
    const size_t n = (size_t)N * N;
    const size_t blocks = (n + NT - 1) / NT;
    for (size_t b = 0; b < blocks; ++b) partials[b] = 0.0;
    for (size_t i = 0; i < n; ++i) {
        W[i] = U[i] - Uk[i];
        partials[i / NT] += W[i] * W[i];
    }
}
void launch_prox(int, const Slot *, int N, const double *c, double *u, hipStream_t) {
    std::memcpy(u, c, (size_t)N * N * sizeof(double));
}
void launch_copy_out(Slot *const *slots, double *out, size_t n, hipStream_t) {
    const Slot &s = *slots[0];
    if (!s.st->outer_done) return;
    const double *src = s.mode == MODE_F64 ? (const double *)s.U[s.st->iters & 1] : s.U64[s.st->outer & 1];
    if (src != out) std::memmove(out, src, n * sizeof(double));
}
void launch_copy_back(Slot *const *slots, int nslots, size_t n, hipStream_t) {
    for (int i = 0; i < nslots; ++i) {
        const Slot &s = *slots[i];
        if (!s.st->outer_done || s.st->status != ST_OK) continue;
        const double *src = s.mode == MODE_F64 ? (const double *)s.U[s.st->iters & 1] : s.U64[s.st->outer & 1];
        std::memmove(const_cast<double *>(s.src), src, n * sizeof(double));
    }
}
}  // namespace rdk

// ------------------------------------------------------------------ scenarios
namespace {

rd_problem ac(int N) {
    rd_problem p{};
    p.nx = p.ny = N;
    p.lx = p.ly = 1.0;
    p.bc = RD_BC_PERIODIC;
    p.op = RD_OP_LAP5;
    p.rx = RD_RX_ALLEN_CAHN;
    p.nz = 0;
    p.diff[0] = 1e-4;
    p.p[0] = 1.0;
    return p;
}

rd_opts opts(double tol, int prec) {
    rd_opts o;
    rd_default_opts(&o);
    o.tol = tol;
    o.precision = prec;
    o.inner_rtol = 1e-3;   // the inner-loop lengths the scenarios expect
    return o;
}

// iterations the residual model needs: the least n with q^n <= tol
int model_iters(double ht, double tol) {
    int n = 0;
    double r = 1.0;
    while (r > tol) {
        r *= model_q(ht);
        ++n;
    }
    return n;
}

double *dalloc(size_t n) {
    void *p = nullptr;
    hipMalloc(&p, n * sizeof(double));
    return (double *)p;
}

bool all_equal(const double *a, size_t n, double v) {
    for (size_t i = 0; i < n; ++i)
        if (a[i] != v) return false;
    return true;
}

void validation() {
    rd_ctx *ctx = nullptr, *other = nullptr;
    CHECK(rd_create(1, &other) == RD_E_INVALID && other == nullptr);
    CHECK(rd_create(0, &ctx) == RD_OK);
    CHECK(rd_create(0, nullptr) == RD_E_INVALID);
    rd_opts o = opts(1e-3, RD_FP64);
    double *u = dalloc(64 * 64), *v = dalloc(64 * 64);
    rd_info info;
    rd_problem p = ac(64);
    p.nx = 48;
    p.ny = 48;
    CHECK(rd_step(ctx, &p, &o, 0.01, u, v, nullptr, &info) == RD_E_INVALID);   // not a power of two
    p = ac(64);
    p.ny = 32;
    CHECK(rd_step(ctx, &p, &o, 0.01, u, v, nullptr, &info) == RD_E_INVALID);   // not square
    p = ac(8192);
    CHECK(rd_step(ctx, &p, &o, 0.01, u, v, nullptr, &info) == RD_E_INVALID);   // too large
    p = ac(64);
    CHECK(rd_step(ctx, &p, &o, 0.0, u, v, nullptr, &info) == RD_E_INVALID);    // h_t <= 0
    CHECK(rd_step(ctx, &p, &o, NAN, u, v, nullptr, &info) == RD_E_INVALID);
    p.rx = RD_RX_CAHN_HILLIARD;                                                  // CH needs BIHARM13
    CHECK(rd_step(ctx, &p, &o, 0.01, u, v, nullptr, &info) == RD_E_INVALID);
    p = ac(64);
    rd_opts bad = o;
    bad.tau_u = 0.0;
    CHECK(rd_step(ctx, &p, &bad, 0.01, u, v, nullptr, &info) == RD_E_INVALID);
    bad = o;
    bad.precision = 7;
    CHECK(rd_step(ctx, &p, &bad, 0.01, u, v, nullptr, &info) == RD_E_INVALID);
    p.op = RD_OP_FCH6;
    p.rx = RD_RX_FCH;
    rd_opts mixed = opts(1e-3, RD_FP32_MIXED);
    CHECK(rd_step(ctx, &p, &mixed, 0.01, u, v, nullptr, &info) == RD_E_INVALID);   // FCH: FP64 only
    CHECK(rd_footprint_bytes(&p, &mixed) == 0);
    p = ac(64);
    CHECK(rd_footprint_bytes(&p, &o) > 6 * 64 * 64 * sizeof(double));
    CHECK(rd_step(nullptr, &p, &o, 0.01, u, v, nullptr, &info) == RD_E_INVALID);
    hipFree(u);
    hipFree(v);
    CHECK(rd_destroy(ctx) == RD_OK);
}

void fp64_steps() {
    rd_ctx *ctx = nullptr;
    rd_create(0, &ctx);
    const int N = 32;
    const size_t n = (size_t)N * N;
    rd_problem p = ac(N);
    const double ht = 0.01, tol = 1e-3;
    const int it = model_iters(ht, tol);
    rd_opts o = opts(tol, RD_FP64);
    double *a = dalloc(n), *b = dalloc(n + 1);
    for (size_t i = 0; i < n; ++i) a[i] = 0.25;
    rd_info info;
    // a chain of steps: out-of-place, alternating buffers (the output binds as the
    // iterate buffer of the previous step's parity), then in place
    double expect = 0.25;
    for (int k = 0; k < 6; ++k) {
        double *in = (k & 1) ? b : a, *out = (k & 1) ? a : b;
        CHECK(rd_step(ctx, &p, &o, ht, in, out, nullptr, &info) == RD_OK);
        expect += it;
        CHECK(info.iters == it && info.status == RD_OK && info.outer == 0);
        CHECK(all_equal(out, n, expect));
    }
    double *cur = a;   // after an even number of steps the state is in a
    for (int k = 0; k < 3; ++k) {
        CHECK(rd_step(ctx, &p, &o, ht, cur, cur, nullptr, &info) == RD_OK);
        expect += it;
        CHECK(all_equal(cur, n, expect));
    }
    // an output that is not 32-byte aligned takes the host-enqueued copy
    CHECK(rd_step(ctx, &p, &o, ht, cur, b + 1, nullptr, &info) == RD_OK);
    CHECK(all_equal(b + 1, n, expect + it));
    // already converged at U_0: zero iterations, the input comes back
    rd_opts loose = opts(2.0, RD_FP64);
    CHECK(rd_step(ctx, &p, &loose, ht, cur, b, nullptr, &info) == RD_OK);
    CHECK(info.iters == 0 && all_equal(b, n, expect));
    // iteration limit
    rd_opts lim = o;
    lim.max_iter = 3;
    CHECK(rd_step(ctx, &p, &lim, ht, cur, b, nullptr, &info) == RD_E_NOCONV);
    CHECK(info.iters == 3 && all_equal(b, n, expect + 3));
    lim.max_iter = 0;
    CHECK(rd_step(ctx, &p, &lim, ht, cur, b, nullptr, &info) == RD_E_NOCONV);
    CHECK(info.iters == 0 && all_equal(b, n, expect));
    // divergence: the residual grows by 3 per iteration; 1e8 is passed after 17
    CHECK(rd_step(ctx, &p, &o, 2.0, cur, b, nullptr, &info) == RD_E_NONFINITE);
    CHECK(info.iters == 17);
    // a long step after short ones: the chunk schedule grows until it ends
    rd_opts tight = opts(1e-30, RD_FP64);
    CHECK(rd_step(ctx, &p, &tight, 0.5, cur, b, nullptr, &info) == RD_OK);
    CHECK(info.iters == model_iters(0.5, 1e-30));
    hipFree(a);
    hipFree(b);
    rd_destroy(ctx);
}

void mixed_steps() {
    rd_ctx *ctx = nullptr;
    rd_create(0, &ctx);
    const int N = 16;
    const size_t n = 2 * (size_t)N * N;
    rd_problem p = ac(N);
    p.rx = RD_RX_SCHNAKENBERG;
    p.diff[1] = 10.0;
    p.p[0] = 0.1;
    p.p[1] = 0.9;
    p.p[2] = 1.0;
    const double ht = 0.01;
    rd_opts o = opts(1e-6, RD_FP32_MIXED);
    double *a = dalloc(n), *b = dalloc(n);
    for (size_t i = 0; i < n; ++i) a[i] = 1.0;
    rd_info info;
    // q = 1/2: each inner loop needs 10 iterations (2^-10 <= 1e-3); the outer norm
    // after 20 is 2^-20 <= 1e-6
    double expect = 1.0;
    for (int k = 0; k < 5; ++k) {
        double *in = (k & 1) ? b : a, *out = (k & 1) ? a : b;
        CHECK(rd_step(ctx, &p, &o, ht, in, out, nullptr, &info) == RD_OK);
        expect += 20;
        CHECK(info.iters == 20 && info.outer == 2 && info.status == RD_OK);
        CHECK(all_equal(out, n, expect));
    }
    rd_opts lim = o;
    lim.max_outer = 1;
    CHECK(rd_step(ctx, &p, &lim, ht, a, a, nullptr, &info) == RD_E_NOCONV);
    CHECK(info.outer == 1 && info.iters == 10);
    hipFree(a);
    hipFree(b);
    rd_destroy(ctx);
}

void serving() {
    rd_ctx *ctx = nullptr;
    rd_create(0, &ctx);
    struct T {
        int N, prec, steps;
        double ht, tol;
        rd_traj *h;
        double *u;
        std::vector<uint64_t> tickets;
    };
    std::vector<T> ts = {{16, RD_FP64, 3, 0.01, 1e-3, nullptr, nullptr, {}},
                         {32, RD_FP32_MIXED, 2, 0.01, 1e-6, nullptr, nullptr, {}},
                         {16, RD_FP64, 4, 0.003, 1e-5, nullptr, nullptr, {}},
                         {32, RD_FP64, 2, 0.5, 1e-4, nullptr, nullptr, {}},
                         {16, RD_FP32_MIXED, 3, 0.01, 1e-6, nullptr, nullptr, {}},
                         {64, RD_FP64, 1, 0.01, 1e-3, nullptr, nullptr, {}}};
    // budget for about two 32^2 workspaces: admission must wait for closes... and
    // never for a lone trajectory
    rd_opts o64 = opts(1e-3, RD_FP64);
    rd_problem p32 = ac(32);
    CHECK(rd_serve_set_budget(ctx, 2 * rd_footprint_bytes(&p32, &o64)) == RD_OK);
    for (T &t : ts) {
        rd_problem p = ac(t.N);
        rd_opts o = opts(t.tol, t.prec);
        t.u = dalloc((size_t)t.N * t.N);
        for (int i = 0; i < t.N * t.N; ++i) t.u[i] = 0.5;
        CHECK(rd_traj_open(ctx, &p, &o, t.u, nullptr, &t.h) == RD_OK);
        for (int k = 0; k < t.steps; ++k) {
            uint64_t tk = 0;
            CHECK(rd_traj_submit(t.h, t.ht, &tk) == RD_OK);
            t.tickets.push_back(tk);
        }
    }
    rd_info info;
    CHECK(rd_poll(ctx, ts[0].tickets[0], &info) == RD_E_BUSY);
    CHECK(rd_poll(ctx, 123456789, &info) == RD_E_INVALID);
    int rounds = 0, closed = 0;
    std::vector<int> done_steps(ts.size(), 0);
    while (closed < (int)ts.size() && rounds < 10000) {
        CHECK(rd_serve_pump(ctx, 0) == RD_OK);
        ++rounds;
        rd_serve_info si;
        rd_serve_stats(ctx, &si);
        CHECK(si.admitted <= 1 || si.resident_bytes <= si.budget_bytes);
        for (size_t i = 0; i < ts.size(); ++i) {
            T &t = ts[i];
            if (!t.h) continue;
            while (done_steps[i] < t.steps && rd_poll(ctx, t.tickets[done_steps[i]], &info) != RD_E_BUSY) {
                const int want = t.prec == RD_FP64 ? model_iters(t.ht, t.tol) : 20;
                CHECK(info.status == RD_OK && info.iters == want);
                ++done_steps[i];
            }
            if (done_steps[i] == t.steps) {
                double *out = dalloc((size_t)t.N * t.N);
                CHECK(rd_traj_read(t.h, out, nullptr) == RD_OK);
                const int per = t.prec == RD_FP64 ? model_iters(t.ht, t.tol) : 20;
                CHECK(all_equal(out, (size_t)t.N * t.N, 0.5 + per * t.steps));
                hipFree(out);
                CHECK(rd_traj_close(t.h) == RD_OK);
                t.h = nullptr;
                ++closed;
            }
        }
    }
    CHECK(closed == (int)ts.size());
    // a closed trajectory's tickets are released
    for (T &t : ts) CHECK(rd_poll(ctx, t.tickets[0], &info) == RD_E_INVALID);
    rd_serve_info si;
    rd_serve_stats(ctx, &si);
    CHECK(si.admitted == 0 && si.resident_bytes == 0 && si.queued == 0 && si.running == 0);
    for (T &t : ts) hipFree(t.u);
    rd_destroy(ctx);
}

// Closing a trajectory with steps still queued drops them: their tickets become
// unknown instead of staying busy, and the other trajectories' steps complete.
void close_with_pending_steps() {
    rd_ctx *ctx = nullptr;
    rd_create(0, &ctx);
    rd_problem p = ac(16);
    rd_opts o = opts(1e-3, RD_FP64);
    double *u = dalloc(256);
    for (int i = 0; i < 256; ++i) u[i] = 0.5;
    rd_traj *a = nullptr, *b = nullptr;
    CHECK(rd_traj_open(ctx, &p, &o, u, nullptr, &a) == RD_OK);
    CHECK(rd_traj_open(ctx, &p, &o, u, nullptr, &b) == RD_OK);
    uint64_t ta[3], tb = 0;
    for (uint64_t &tk : ta) CHECK(rd_traj_submit(a, 0.01, &tk) == RD_OK);
    CHECK(rd_traj_submit(b, 0.01, &tb) == RD_OK);
    rd_info info;
    CHECK(rd_serve_pump(ctx, 0) == RD_OK);   // a's first step and b's step start
    double *mid = dalloc(256);
    CHECK(rd_traj_read(b, mid, nullptr) == RD_OK);   // waits for b's round, if in flight
    hipFree(mid);
    CHECK(rd_traj_close(a) == RD_OK);
    for (uint64_t tk : ta) CHECK(rd_poll(ctx, tk, &info) == RD_E_INVALID);
    for (int k = 0; k < 100 && rd_poll(ctx, tb, &info) == RD_E_BUSY; ++k) CHECK(rd_serve_pump(ctx, 0) == RD_OK);
    CHECK(rd_poll(ctx, tb, &info) == RD_OK && info.iters == model_iters(0.01, 1e-3));
    rd_serve_info si;
    rd_serve_stats(ctx, &si);
    CHECK(si.queued == 0 && si.running == 0);
    CHECK(rd_traj_close(b) == RD_OK);
    hipFree(u);
    rd_destroy(ctx);
}

// A served step that stops at the iteration limit reports RD_E_NOCONV and leaves the
// trajectory's state; the next step of a trajectory with room to converge starts from it.
void failed_step_leaves_state() {
    rd_ctx *ctx = nullptr;
    rd_create(0, &ctx);
    rd_problem p = ac(16);
    rd_opts tight = opts(1e-3, RD_FP64);
    tight.max_iter = 2;
    double *u = dalloc(256);
    for (int i = 0; i < 256; ++i) u[i] = 0.5;
    rd_traj *t = nullptr;
    CHECK(rd_traj_open(ctx, &p, &tight, u, nullptr, &t) == RD_OK);
    uint64_t tk = 0;
    CHECK(rd_traj_submit(t, 0.01, &tk) == RD_OK);
    rd_info info;
    for (int k = 0; k < 100 && rd_poll(ctx, tk, &info) == RD_E_BUSY; ++k) CHECK(rd_serve_pump(ctx, 0) == RD_OK);
    CHECK(rd_poll(ctx, tk, &info) == RD_E_NOCONV && info.status == RD_E_NOCONV);
    double *out = dalloc(256);
    CHECK(rd_traj_read(t, out, nullptr) == RD_OK && all_equal(out, 256, 0.5));
    CHECK(rd_traj_close(t) == RD_OK);
    // the same start, with room to converge: the model's iterate gains 1 per iteration
    rd_opts o = opts(1e-3, RD_FP64);
    CHECK(rd_traj_open(ctx, &p, &o, out, nullptr, &t) == RD_OK);
    CHECK(rd_traj_submit(t, 0.01, &tk) == RD_OK);
    for (int k = 0; k < 100 && rd_poll(ctx, tk, &info) == RD_E_BUSY; ++k) CHECK(rd_serve_pump(ctx, 0) == RD_OK);
    CHECK(rd_poll(ctx, tk, &info) == RD_OK);
    CHECK(rd_traj_read(t, out, nullptr) == RD_OK && all_equal(out, 256, 0.5 + model_iters(0.01, 1e-3)));
    CHECK(rd_traj_close(t) == RD_OK);
    hipFree(out);
    hipFree(u);
    rd_destroy(ctx);
}

void adaptive() {
    rd_adapt a{};
    a.ht0 = 0.02;
    a.eta = 0.5;
    a.n_hi = 12;
    a.n_lo = 4;
    a.ht_min = 1e-9;
    a.max_rejects = 5;
    double nx = 0;
    int32_t acc = 0;
    CHECK(rd_adapt_next(&a, 0.01, 20, RD_OK, &nx, &acc) == RD_OK && acc == 1 && nx == 0.005);
    CHECK(rd_adapt_next(&a, 0.01, 2, RD_OK, &nx, &acc) == RD_OK && acc == 1 && nx == 0.02);
    CHECK(rd_adapt_next(&a, 0.02, 2, RD_OK, &nx, &acc) == RD_OK && nx == 0.02);   // capped at ht0
    CHECK(rd_adapt_next(&a, 0.01, 8, RD_OK, &nx, &acc) == RD_OK && nx == 0.01);
    CHECK(rd_adapt_next(&a, 0.01, 8, RD_E_NOCONV, &nx, &acc) == RD_OK && acc == 0 && nx == 0.005);
    rd_adapt bad = a;
    bad.eta = 1.0;
    CHECK(rd_adapt_next(&bad, 0.01, 8, RD_OK, &nx, &acc) == RD_E_INVALID);
    // a run: q(h) makes large steps take many iterations, so the rule settles
    rd_ctx *ctx = nullptr;
    rd_create(0, &ctx);
    const int N = 16;
    rd_problem p = ac(N);
    rd_opts o = opts(1e-3, RD_FP64);
    double *u = dalloc((size_t)N * N);
    for (int i = 0; i < N * N; ++i) u[i] = 0.0;
    rd_adapt_info info;
    double th[64];
    int32_t ti[64], tok[64];
    CHECK(rd_advance(ctx, &p, &o, &a, 0.0, 0.1, u, nullptr, &info, th, ti, tok, 64) == RD_OK);
    CHECK(std::fabs(info.t - 0.1) < 1e-12 && info.accepted > 0 && info.shrinks > 0);
    CHECK(all_equal(u, (size_t)N * N, (double)info.pdhg_iters));   // every step was accepted
    // divergence at h_t >= 1: rejected, shrunk, then accepted
    a.ht0 = 1.5;
    CHECK(rd_advance(ctx, &p, &o, &a, 0.0, 1.5, u, nullptr, &info, th, ti, tok, 64) == RD_OK);
    CHECK(info.rejected >= 1 && tok[0] == 0);
    hipFree(u);
    rd_destroy(ctx);
}

// A column pass (3-D: forward y pass) reads the State in every workgroup while its
// extra workgroup writes the decision of the preceding row pass, so workgroups may
// see the State before or after it.  The transforming workgroups branch only on
// outer_done; the decision may change it only from 0 to 1, and then nothing reads
// the pass's output.  Checked here over random States and residuals.
void column_pass_race_invariant() {
    unsigned x = 12345;
    auto rnd = [&]() { x = x * 1103515245u + 12345u; return (x >> 8) & 0xffff; };
    const StopRule rule{1e-6, 1e-3, 50, 4};
    for (int t = 0; t < 200000; ++t) {
        // reachable States: FP64 keeps outer_done == done; in the mixed path a
        // finished step has finished its inner loop
        State in{};
        in.done = rnd() & 1;
        in.outer_done = in.done && (rnd() & 1) ? 1 : 0;
        in.iters = rnd() % 60;
        in.total_iters = in.iters + rnd() % 100;
        in.outer = rnd() % 5;
        in.inner_best_it = rnd() % (in.iters + 1);
        in.res0 = 1.0;
        in.inner_target = 1e-3 * (rnd() % 3);
        in.inner_best = 1e-2 * (1 + rnd() % 50);
        in.outer_res = 1e-3 * (1 + rnd() % 100);
        const double res = (rnd() % 17 == 0) ? NAN : 1e-8 * (rnd() % 200000);
        if (!skip(K_ITER64, in) && in.outer_done == in.done) {
            const State out = decide<K_ITER64>(in, rule, res, 0.0);
            CHECK(out.outer_done == in.outer_done || out.outer_done == 1);
        }
        if (!skip(K_MIXED, in)) {
            const State out = decide<K_MIXED>(in, rule, res, 0.0);
            CHECK(out.outer_done == in.outer_done || out.outer_done == 1);
        }
    }
}

// rd_step_noalloc: the results and counts of rd_step, on the scratch array, with no
// allocation (the stub's live-allocation count does not move during the calls);
// problems beyond the array are refused.
void noalloc_steps() {
    rd_ctx *ctx = nullptr;
    rd_create(0, &ctx);
    for (int prec : {RD_FP64, RD_FP32_MIXED}) {
        for (int N : {256, 32}) {
            const size_t n = (size_t)N * N;
            rd_problem p = ac(N);
            rd_opts o = opts(prec == RD_FP64 ? 1e-3 : 1e-6, prec);
            double *u = dalloc(n), *a = dalloc(n), *b = dalloc(n + 1);
            for (size_t i = 0; i < n; ++i) u[i] = 0.125;
            rd_info ia, ib;
            CHECK(rd_step(ctx, &p, &o, 0.01, u, a, nullptr, &ia) == RD_OK);
            const long live = hipstub::live_allocs();
            CHECK(rd_step_noalloc(ctx, &p, &o, 0.01, u, b, nullptr, &ib) == RD_OK);
            CHECK(rd_step_noalloc(ctx, &p, &o, 0.01, u, b + 1, nullptr, &ib) == RD_OK);   // unaligned output
            CHECK(rd_step_noalloc(ctx, &p, &o, 0.01, u, u, nullptr, &ib) == RD_OK);       // in place
            CHECK(hipstub::live_allocs() == live);
            CHECK(ia.iters == ib.iters && ia.outer == ib.outer && ia.status == ib.status);
            CHECK(std::memcmp(a, b + 1, n * sizeof(double)) == 0 && std::memcmp(a, u, n * sizeof(double)) == 0);
            hipFree(u);
            hipFree(a);
            hipFree(b);
        }
    }
    rd_problem big = ac(2048);
    rd_opts o = opts(1e-3, RD_FP64);
    double *u = dalloc(16);
    rd_info info;
    CHECK(rd_step_noalloc(ctx, &big, &o, 0.01, u, u, nullptr, &info) == RD_E_NOMEM);
    big = ac(1024);
    big.rx = RD_RX_SCHNAKENBERG;
    big.diff[1] = 10.0;
    CHECK(rd_step_noalloc(ctx, &big, &o, 0.01, u, u, nullptr, &info) == RD_E_NOMEM);
    hipFree(u);
    rd_destroy(ctx);
}

void teardown_returns_everything() {
    const long base = hipstub::live_allocs();
    for (int r = 0; r < 20; ++r) {
        rd_ctx *ctx = nullptr;
        rd_create(0, &ctx);
        rd_problem p = ac(16);
        rd_opts o = opts(1e-3, r & 1 ? RD_FP32_MIXED : RD_FP64);
        double *u = dalloc(256);
        rd_info info;
        rd_step(ctx, &p, &o, 0.01, u, u, nullptr, &info);
        rd_traj *t = nullptr;
        rd_traj_open(ctx, &p, &o, u, nullptr, &t);
        uint64_t tk;
        rd_traj_submit(t, 0.01, &tk);
        for (int k = 0; k < 20 && rd_poll(ctx, tk, &info) == RD_E_BUSY; ++k) rd_serve_pump(ctx, 0);
        if (r % 3 == 0) rd_traj_close(t);   // the others are freed by rd_destroy
        hipFree(u);
        rd_destroy(ctx);
    }
    CHECK(hipstub::live_allocs() == base);
    CHECK(hipstub::live_streams() == 0);
}

}  // namespace

int main() {
    validation();
    fp64_steps();
    mixed_steps();
    serving();
    close_with_pending_steps();
    failed_step_leaves_state();
    adaptive();
    column_pass_race_invariant();
    noalloc_steps();
    teardown_returns_everything();
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
