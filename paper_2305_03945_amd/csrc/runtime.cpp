// Host runtime of librdpdhg: argument validation, per-size tables, workspaces,
// the launch schedule of one implicit step, the kernel-level entry points and
// the continuous-batching serving loop.  Implements include/rd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/rd.h"
#include "registry.h"

using namespace rdk;

namespace {

#define RD_CHECK(call)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            if (std::getenv("RD_LOG"))                                                       \
                std::fprintf(stderr, "[rd] %s:%d %s -> %s\n", __FILE__, __LINE__, #call,   \
                             hipGetErrorString(e_));                                         \
            return RD_E_DEVICE;                                                              \
        }                                                                                    \
    } while (0)

std::once_flag g_register_once;
void register_all() {
    register_logn_4();
    register_logn_5();
    register_logn_6();
    register_logn_7();
    register_logn_8();
    register_logn_9();
    register_logn_10();
    register_logn_11();
    register_logn_12();
}

// ---------------------------------------------------------------- problem description
struct Desc {
    int N = 0, logN = 0, C = 1, bc = 0, eq = 0, mode = 0;
    int dim = 2;          // 2: N x N grid; 3: N x N x N grid (7-point Laplacian)
    size_t pts = 0;       // points per component, N^dim
    int rows = 0;         // x-rows per component, N^(dim-1)
    double h = 0;
};

int ilog2_exact(int n) {
    if (n <= 0 || (n & (n - 1))) return -1;
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

rd_status describe(const rd_problem *p, Desc &d) {
    if (!p) return RD_E_INVALID;
    if (p->nx != p->ny || !(p->lx > 0.0) || p->lx != p->ly) return RD_E_INVALID;
    const int l = ilog2_exact(p->nx);
    if (l < LOGN_MIN || l > LOGN_MAX) return RD_E_INVALID;
    if (p->bc != RD_BC_PERIODIC && p->bc != RD_BC_NEUMANN) return RD_E_INVALID;
    d.N = p->nx;
    d.logN = l;
    d.bc = p->bc == RD_BC_PERIODIC ? BC_P : BC_N;
    d.h = p->lx / p->nx;
    d.dim = 2;
    if (p->nz > 1) {
        // 3-D: a cube of N^3 points, 7-point Laplacian equations only
        if (p->nz != p->nx || l > LOGN3_MAX) return RD_E_INVALID;
        if (p->op != RD_OP_LAP5) return RD_E_INVALID;
        d.dim = 3;
    } else if (p->nz < 0) {
        return RD_E_INVALID;
    }
    d.pts = (size_t)d.N * d.N * (d.dim == 3 ? d.N : 1);
    d.rows = d.N * (d.dim == 3 ? d.N : 1);
    if (p->op == RD_OP_LAP5 && (p->rx == RD_RX_NONE || p->rx == RD_RX_ALLEN_CAHN)) {
        d.eq = EQ_LAP5;
        d.C = 1;
    } else if (p->op == RD_OP_BIHARM13 && (p->rx == RD_RX_NONE || p->rx == RD_RX_CAHN_HILLIARD)) {
        d.eq = EQ_BIH;
        d.C = 1;
    } else if (p->op == RD_OP_FCH6 && p->rx == RD_RX_FCH) {
        d.eq = EQ_FCH;
        d.C = 1;
    } else if (p->op == RD_OP_LAP5 && p->rx == RD_RX_SCHNAKENBERG) {
        d.eq = EQ_SCHNAK;
        d.C = 2;
    } else {
        return RD_E_INVALID;
    }
    if (!(p->diff[0] >= 0.0) || (d.C == 2 && !(p->diff[1] >= 0.0))) return RD_E_INVALID;
    return RD_OK;
}

const KSet &kset(int mode, const Desc &d) {
    return d.dim == 3 ? g_kernels3[mode][d.logN][d.bc][d.eq] : g_kernels[mode][d.logN][d.bc][d.eq];
}

rd_status check_opts(const rd_opts *o) {
    if (!o) return RD_E_INVALID;
    if (!(o->tol >= 0.0) || o->max_iter < 0 || o->max_outer < 0) return RD_E_INVALID;
    if (!(o->tau_u > 0.0) || !(o->tau_p > 0.0) || !(o->omega >= 0.0)) return RD_E_INVALID;
    if (o->precision != RD_FP64 && o->precision != RD_FP32_MIXED) return RD_E_INVALID;
    if (o->init != RD_INIT_PREV && o->init != RD_INIT_PROX) return RD_E_INVALID;
    if (o->precision == RD_FP32_MIXED && !(o->inner_rtol > 0.0)) return RD_E_INVALID;
    return RD_OK;
}

// ---------------------------------------------------------------- per-size tables
struct Tables {
    double *eig = nullptr;            // s_k (FP64)
    void *tw[2] = {nullptr, nullptr};  // [mode]: FFT twiddles in the mode's transform type
    void *twd[2] = {nullptr, nullptr}; // [mode]: DCT twiddles
};

// ---------------------------------------------------------------- workspace of one slot
struct Workspace {
    int N = 0, C = 0, mode = 0, logN = 0, nblk = 0, dim = 2;
    size_t pts = 0;
    size_t bytes = 0;
    std::vector<void *> allocs;
    Slot *slot_dev = nullptr;     // device copy of the slot
    Slot **slot_list_dev = nullptr; // device array {slot_dev}
    Slot *slot_host = nullptr;    // pinned staging
    State *st_host = nullptr;     // pinned readback
    Slot proto{};                 // pointers filled at allocation
    // iteration launches the last two steps on this workspace used (FP64: their
    // iterations; mixed: their inner iterations plus one per outer update)
    int last_iters = 0, prev_iters = 0;
    int last_parity = -1;   // index of the iterate buffer the previous step ended in
};

// Record the length of a finished step for the next step's schedule.  A mixed
// step uses one iteration launch per inner iteration and one per outer update
// (the row pass of that launch makes the update).
void remember_step(Workspace &w, const State &s) {
    w.prev_iters = w.last_iters;
    w.last_iters = w.mode == MODE_F64 ? s.iters : s.total_iters + s.outer;
    w.last_parity = w.mode == MODE_F64 ? (s.iters & 1) : (s.outer & 1);
}

// Iterations the first chunk of a step enqueues: what the previous step used,
// plus its growth over the step before (one more while only one step is known).
// Along a trajectory consecutive steps mostly need the same count (2048^2
// Allen-Cahn: 195 of 199 steps equal, the others fewer), and an iteration
// enqueued beyond the end costs a wasted column pass and three skipped
// launches (about 20 us at 2048^2), while one missing costs a host round trip.
int first_chunk(const Workspace &w) {
    if (w.last_iters <= 0) return w.mode == MODE_F64 ? 8 : 16;
    if (w.prev_iters <= 0) return w.last_iters + 1;
    return w.last_iters + std::max(0, w.last_iters - w.prev_iters);
}

// pts: points per component (N^2 or N^3)
size_t field_bytes(size_t pts, int C, size_t elem) { return (size_t)C * pts * elem; }

// rows: x-rows per component (N or N^2)
size_t workspace_bytes(size_t pts, int rows, int C, int mode, int rows_per_block) {
    const size_t nblk = rows_per_block > 0 ? (size_t)rows / rows_per_block : (size_t)rows / 2;
    const size_t N = pts;
    size_t b = 0;
    if (mode == MODE_F64) {
        b += 5 * field_bytes(N, C, 8);   // U[2], P, Pt, S
        b += field_bytes(N, C, 8);       // Uk
    } else {
        b += 4 * field_bytes(N, C, 4);   // e[2], P, Pt
        b += field_bytes(N, C, 4);       // S
        b += 2 * field_bytes(N, C, 4);   // r32, Ub32
        b += 3 * field_bytes(N, C, 8);   // U64[2], Uk
    }
    b += nblk * 2 * C * sizeof(double) + sizeof(State) + sizeof(Slot) + sizeof(Slot *) + 4096;
    return b;
}

// Serving batch groups: steps that share a key run in one launch per kernel.
struct GroupKey {
    int mode, logN, bc, eq, dim;
    bool operator<(const GroupKey &o) const {
        return std::tie(mode, logN, bc, eq, dim) < std::tie(o.mode, o.logN, o.bc, o.eq, o.dim);
    }
};

// Device slot-pointer list of one (group, role): role 0 for the init launch of
// starting steps, role 1 for the iteration round.  A list is rewritten only in a
// later pump round, after the stream that read it was synchronised.
struct BatchBuffers {
    Slot **dev = nullptr;
    Slot **host = nullptr;
    int cap = 0;
};
struct Ticket {
    rd_info info{};
    bool done = false;
};

struct Traj;

// A batch group's round: its own stream (default priority), so that groups of
// different shapes overlap on the device and each finishes on its own; the event
// recorded after the round's work; the trajectories the round advances.  A group
// has at most one round in flight, and its slot lists are rewritten only when
// none is.
struct GroupRound {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool in_flight = false;
    std::vector<Traj *> trajs;
};

struct Ctx {
    int device = 0;
    std::map<std::tuple<int, int, uint64_t>, Tables> tables;  // (N, bc, bits of h)
    std::map<std::tuple<int, int, int, int>, std::unique_ptr<Workspace>> step_ws;  // (N, C, mode, dim)
    // scratch for kernel-level entry points
    Slot *scratch_slot_dev = nullptr;
    Slot *scratch_slot_host = nullptr;
    double *scratch_partials = nullptr;
    size_t scratch_partials_n = 0;
    std::vector<double> host_partials;
    // serving
    size_t budget = 0, resident = 0;
    uint64_t next_ticket = 1;
    std::map<uint64_t, Ticket> tickets;
    std::vector<Traj *> trajs;
    std::deque<Traj *> admit_queue;
    std::map<std::pair<GroupKey, int>, BatchBuffers> batch;
    std::map<GroupKey, GroupRound> rounds;
};

struct PendingStep {
    uint64_t ticket;
    double ht;
};

struct Traj {
    Ctx *ctx = nullptr;
    rd_problem prob{};
    rd_opts opts{};
    Desc d{};
    double *u = nullptr;                 // resident state U^k (FP64)
    std::unique_ptr<Workspace> ws;       // present once admitted
    std::deque<PendingStep> pending;
    std::vector<uint64_t> tickets;       // every ticket of this trajectory; released at close
    bool running = false;
    uint64_t running_ticket = 0;
    int issued = 0;                      // iterations launched for the running step
    bool queued_for_admission = false;
};

rd_status dmalloc(Workspace &w, void **p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) return RD_E_NOMEM;
    w.allocs.push_back(*p);
    return RD_OK;
}

void free_workspace(Workspace *w) {
    if (!w) return;
    for (void *p : w->allocs) (void)hipFree(p);
    w->allocs.clear();
    if (w->slot_host) (void)hipHostFree(w->slot_host);
    if (w->st_host) (void)hipHostFree(w->st_host);
    w->slot_host = nullptr;
    w->st_host = nullptr;
}

rd_status make_workspace(const Desc &d, int mode, std::unique_ptr<Workspace> &out) {
    auto w = std::make_unique<Workspace>();
    const int C = d.C;
    const size_t N = d.pts;   // the field sizes below are per point
    w->N = d.N;
    w->C = C;
    w->mode = mode;
    w->logN = d.logN;
    w->dim = d.dim;
    w->pts = d.pts;
    const KSet &k = kset(mode, d);
    if (!k.init) return RD_E_INVALID;
    w->nblk = d.rows / k.rows_per_block;
    w->bytes = workspace_bytes(d.pts, d.rows, C, mode, k.rows_per_block);
    Slot &s = w->proto;
    std::memset(&s, 0, sizeof(Slot));
    rd_status r;
    const size_t te = mode == MODE_F64 ? 8 : 4;
#define ALLOC(ptr, bytes)                                          \
    do {                                                           \
        void *p_ = nullptr;                                        \
        if ((r = dmalloc(*w, &p_, (bytes))) != RD_OK) {            \
            free_workspace(w.get());                               \
            return r;                                              \
        }                                                          \
        ptr = decltype(ptr)(p_);                                   \
    } while (0)
    ALLOC(s.U[0], field_bytes(N, C, te));
    ALLOC(s.U[1], field_bytes(N, C, te));
    ALLOC(s.P, field_bytes(N, C, te));
    ALLOC(s.Pt, field_bytes(N, C, te));
    ALLOC(s.S, field_bytes(N, C, te));
    ALLOC(s.Uk, field_bytes(N, C, 8));
    if (mode == MODE_MIXED) {
        ALLOC(s.U64[0], field_bytes(N, C, 8));
        ALLOC(s.U64[1], field_bytes(N, C, 8));
        ALLOC(s.r32, field_bytes(N, C, 4));
        ALLOC(s.Ub32, field_bytes(N, C, 4));
    }
    ALLOC(s.partials, (size_t)w->nblk * 2 * C * sizeof(double));
    ALLOC(s.st, sizeof(State));
    ALLOC(w->slot_dev, sizeof(Slot));
    ALLOC(w->slot_list_dev, sizeof(Slot *));
#undef ALLOC
    if (hipHostMalloc((void **)&w->slot_host, sizeof(Slot), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&w->st_host, sizeof(State), hipHostMallocDefault) != hipSuccess) {
        free_workspace(w.get());
        return RD_E_NOMEM;
    }
    if (hipMemset(s.st, 0, sizeof(State)) != hipSuccess ||
        hipMemcpy(w->slot_list_dev, &w->slot_dev, sizeof(Slot *), hipMemcpyHostToDevice) != hipSuccess) {
        free_workspace(w.get());
        return RD_E_DEVICE;
    }
    out = std::move(w);
    return RD_OK;
}

// eig: N doubles; tw, twd: 2N doubles (complex, re/im interleaved).
void fill_tables_host(int N, int bc, double h, double *eig, double *tw, double *twd) {
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < N; ++k) {
        const long double arg = (bc == BC_P) ? pi * k / N : pi * k / (2.0L * N);
        const long double sn = std::sin(arg);
        eig[k] = (double)(4.0L / ((long double)h * h) * sn * sn);
        const long double a = 2.0L * pi * k / N;
        tw[2 * k] = (double)std::cos(a);
        tw[2 * k + 1] = (double)(-std::sin(a));
        const long double b = pi * k / (2.0L * N);
        twd[2 * k] = (double)std::cos(b);
        twd[2 * k + 1] = (double)(-std::sin(b));
    }
}

rd_status get_tables(Ctx *c, int N, int bc, double h, Tables *&out) {
    uint64_t hb;
    std::memcpy(&hb, &h, sizeof(hb));
    auto key = std::make_tuple(N, bc, hb);
    auto it = c->tables.find(key);
    if (it != c->tables.end()) {
        out = &it->second;
        return RD_OK;
    }
    std::vector<double> eig(N), tw(2 * N), twd(2 * N);
    fill_tables_host(N, bc, h, eig.data(), tw.data(), twd.data());
    std::vector<float> tw32(tw.begin(), tw.end()), twd32(twd.begin(), twd.end());
    Tables t;
    RD_CHECK(hipMalloc((void **)&t.eig, N * sizeof(double)));
    RD_CHECK(hipMalloc(&t.tw[0], 2 * N * sizeof(double)));
    RD_CHECK(hipMalloc(&t.twd[0], 2 * N * sizeof(double)));
    RD_CHECK(hipMalloc(&t.tw[1], 2 * N * sizeof(float)));
    RD_CHECK(hipMalloc(&t.twd[1], 2 * N * sizeof(float)));
    RD_CHECK(hipMemcpy(t.eig, eig.data(), N * sizeof(double), hipMemcpyHostToDevice));
    RD_CHECK(hipMemcpy(t.tw[0], tw.data(), 2 * N * sizeof(double), hipMemcpyHostToDevice));
    RD_CHECK(hipMemcpy(t.twd[0], twd.data(), 2 * N * sizeof(double), hipMemcpyHostToDevice));
    RD_CHECK(hipMemcpy(t.tw[1], tw32.data(), 2 * N * sizeof(float), hipMemcpyHostToDevice));
    RD_CHECK(hipMemcpy(t.twd[1], twd32.data(), 2 * N * sizeof(float), hipMemcpyHostToDevice));
    out = &(c->tables[key] = t);
    return RD_OK;
}

// Fill the parameter part of a slot from the problem and options.
void fill_params(Slot &s, const rd_problem *p, const rd_opts *o, const Desc &d, double ht) {
    s.N = d.N;
    s.ncomp = d.C;
    s.bc = d.bc;
    s.eq = d.eq;
    s.mode = o ? (o->precision == RD_FP32_MIXED ? MODE_MIXED : MODE_F64) : MODE_F64;
    s.max_iter = o ? o->max_iter : 0;
    s.max_outer = o ? o->max_outer : 0;
    s.init = o ? o->init : 0;
    s.ht = ht;
    s.h = d.h;
    s.inv_h2 = 1.0 / (d.h * d.h);
    s.inv_h4 = s.inv_h2 * s.inv_h2;
    s.diff[0] = p->diff[0];
    s.diff[1] = d.C == 2 ? p->diff[1] : 0.0;
    s.b = 0.0;
    s.sa = s.sb = 0.0;
    s.kappa = 0.0;
    if (p->rx == RD_RX_ALLEN_CAHN || p->rx == RD_RX_CAHN_HILLIARD) s.b = p->p[0];
    if (p->rx == RD_RX_SCHNAKENBERG) {
        s.sa = p->p[0];
        s.sb = p->p[1];
        s.kappa = p->p[2];
    }
    if (o) {
        s.tau_u = o->tau_u;
        s.tau_p = o->tau_p;
        s.omega = o->omega;
        s.tol = o->tol;
        s.inner_rtol = o->inner_rtol;
    }
    // G = (I - alpha Lap + beta Lap^2 - gamma Lap^3)^2 per component
    for (int c = 0; c < 2; ++c) {
        s.alpha[c] = 0.0;
        s.beta[c] = 0.0;
        s.gamma[c] = 0.0;
    }
    if (d.eq == EQ_LAP5) s.alpha[0] = p->diff[0] * ht;
    else if (d.eq == EQ_BIH) s.beta[0] = p->diff[0] * ht;
    else if (d.eq == EQ_FCH) {
        // Sec. 3.3: G = (I - h_t eps^2 Lap (eps^2 Lap - (2 - eps^2)) Lap)^2, eps^2 = diff[0]
        const double e2 = p->diff[0];
        s.beta[0] = ht * e2 * (2.0 - e2);
        s.gamma[0] = ht * e2 * e2;
    } else {
        s.alpha[0] = p->diff[0] * ht;
        s.alpha[1] = p->diff[1] * ht;
    }
}

void bind_workspace(Slot &s, const Workspace &w, const Tables &t) {
    const Slot &q = w.proto;
    for (int i = 0; i < 2; ++i) {
        s.U[i] = q.U[i];
        s.U64[i] = q.U64[i];
    }
    s.P = q.P;
    s.Pt = q.Pt;
    s.S = q.S;
    s.Uk = q.Uk;
    s.r32 = q.r32;
    s.Ub32 = q.Ub32;
    s.partials = q.partials;
    s.st = q.st;
    s.nblk_rows = w.nblk;
    s.eig = t.eig;
    s.tw = t.tw[w.mode];
    s.twd = t.twd[w.mode];
}

// Launch schedule of one step, or of a batch of running slots of one key.
// `slots`: device array of nslots Slot pointers.  Each call enqueues one chunk
// of `iters` iterations: PDHG iterations (FP64), or mixed iterations whose row
// pass makes the FP64 outer update instead when the inner loop has stopped.
// Finished slots turn them into no-ops.  Every chunk starts after a decided row
// pass (the initial pass with its k_finalize, or the previous chunk's final
// k_finalize); inside it, each column pass (3-D: forward y pass) takes the
// decision of the row pass before it, and the chunk ends with a k_finalize so
// that the host sees a decided State.
void enqueue_round(const KSet &k, Slot *const *slots, int nslots, int iters, hipStream_t st) {
    if (k.dim == 3) {
        for (int i = 0; i < iters; ++i) {
            (i == 0 ? k.yfwd : k.yfwd_fin)(slots, nslots, st, nullptr);
            k.zsym(slots, nslots, st, nullptr);
            k.yinv(slots, nslots, st, nullptr);
            k.rowinv(slots, nslots, st, nullptr);
            k.upd(slots, nslots, st, nullptr);
            k.rowfwd(slots, nslots, st, nullptr);
        }
        k.fin(slots, nslots, st, nullptr);
        return;
    }
    for (int i = 0; i < iters; ++i) {
        (i == 0 ? k.cols : k.cols_fin)(slots, nslots, st, nullptr);
        k.rowinv(slots, nslots, st, nullptr);
        k.upd(slots, nslots, st, nullptr);
        k.rowfwd(slots, nslots, st, nullptr);
    }
    k.fin(slots, nslots, st, nullptr);
}

void info_from_state(const State &s, int mode, rd_info *info) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->iters = mode == MODE_F64 ? s.iters : s.total_iters;
    info->outer = mode == MODE_F64 ? 0 : s.outer;
    info->residual_l2 = mode == MODE_F64 ? s.res : s.outer_res;
    info->residual0 = s.res0;
    info->mass_drift = s.mass;
    info->status = s.status;
}

const void *final_buffer(const Workspace &w, const State &s) {
    if (w.mode == MODE_F64) return w.proto.U[s.iters & 1];
    return w.proto.U64[s.outer & 1];
}

rd_status get_step_workspace(Ctx *c, const Desc &d, int mode, Workspace *&out) {
    auto key = std::make_tuple(d.N, d.C, mode, d.dim);
    auto it = c->step_ws.find(key);
    if (it != c->step_ws.end()) {
        // a workspace is reusable across equations of the same shape; the
        // row-block count depends only on (N, C, mode)
        out = it->second.get();
        return RD_OK;
    }
    std::unique_ptr<Workspace> w;
    rd_status r = make_workspace(d, mode, w);
    if (r != RD_OK) return r;
    out = w.get();
    c->step_ws[key] = std::move(w);
    return RD_OK;
}

// Run one step to completion on the workspace's single slot.  out: nullptr, or a
// 32-byte aligned buffer of nout doubles that receives the result on the device
// once the step has finished (a copy enqueued after every chunk, a no-op until
// then), so that a finished step needs no further launch after the host's wait.
rd_status run_step(Ctx *c, Workspace &w, const KSet &k, hipStream_t st, int max_iter, int max_outer,
                   double *out = nullptr, size_t nout = 0) {
    Slot *const *slots = w.slot_list_dev;
    if (k.step_wg) {
        // small grid: the whole step is one launch
        k.step_wg(slots, 1, st, nullptr);
        if (out) launch_copy_out(slots, out, nout, st);
        RD_CHECK(hipGetLastError());
        RD_CHECK(hipMemcpyAsync(w.st_host, w.proto.st, sizeof(State), hipMemcpyDeviceToHost, st));
        RD_CHECK(hipStreamSynchronize(st));
        remember_step(w, *w.st_host);
        (void)c;
        (void)max_iter;
        (void)max_outer;
        return RD_OK;
    }
    k.init(slots, 1, st, nullptr);
    RD_CHECK(hipGetLastError());
    int issued = 0, rounds = 0;
    while (true) {
        int iters = rounds == 0 ? first_chunk(w) : std::max(4, issued / 4);
        if (w.mode == MODE_F64 && max_iter - issued + 1 < iters) iters = std::max(1, max_iter - issued + 1);
        enqueue_round(k, slots, 1, iters, st);
        if (out) launch_copy_out(slots, out, nout, st);
        RD_CHECK(hipGetLastError());
        issued += iters;
        ++rounds;
        RD_CHECK(hipMemcpyAsync(w.st_host, w.proto.st, sizeof(State), hipMemcpyDeviceToHost, st));
        RD_CHECK(hipStreamSynchronize(st));
        const State &s = *w.st_host;
        const bool finished = w.mode == MODE_F64 ? s.done != 0 : s.outer_done != 0;
        if (finished) break;
        // The device enforces max_iter / max_outer; this bound only guards
        // against a host-side schedule that never reaches them.
        const long cap = w.mode == MODE_F64 ? (long)max_iter + 8
                                            : (long)(max_outer + 1) * (long)(max_iter + 2) + 16;
        if (issued > cap + 64) return RD_E_DEVICE;
    }
    remember_step(w, *w.st_host);
    (void)c;
    return RD_OK;
}

// ---------------------------------------------------------------- allocation-free steps
// rd_step_noalloc runs the kernels of rd_step on a workspace carved from the
// device scratch array of kernels_misc.hip.  Per device: the array's address
// (taken once, by rd_create, with the device current) and host-side staging that
// lives in static storage, so that a call allocates nothing.  Calls that overlap
// on one device share all of it and race.
constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr int NOALLOC_MAX_N = 1024;
struct NoAllocDevice {
    char *base = nullptr;        // device address of the scratch array
    Slot slot{};                 // host staging of the slot
    Slot *list = nullptr;        // host staging of the one-entry slot list
    State st{};                  // host staging of the State (zeroed) and its readback
    double eig[NOALLOC_MAX_N], tw[2 * NOALLOC_MAX_N], twd[2 * NOALLOC_MAX_N];
    float tw32[2 * NOALLOC_MAX_N], twd32[2 * NOALLOC_MAX_N];
    int last_iters = 0, prev_iters = 0;   // schedule history, as a Workspace keeps it
};
NoAllocDevice g_noalloc[NOALLOC_MAX_DEVICES];
std::mutex g_noalloc_mu;

rd_status noalloc_setup(int device) {
    if (device >= NOALLOC_MAX_DEVICES) return RD_OK;   // such devices serve rd_step only
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc[device].base) return RD_OK;
    void *p = nullptr;
    const hipError_t e = noalloc_scratch_address(&p);
    if (e != hipSuccess || !p) {
        if (std::getenv("RD_LOG"))
            std::fprintf(stderr, "[rd] scratch address on device %d: %s\n", device, hipGetErrorString(e));
        return RD_E_DEVICE;
    }
    g_noalloc[device].base = (char *)p;
    return RD_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char *rd_status_str(rd_status s) {
    switch (s) {
    case RD_OK: return "ok";
    case RD_E_INVALID: return "invalid argument";
    case RD_E_NOCONV: return "iteration limit reached";
    case RD_E_NONFINITE: return "residual non-finite or diverging";
    case RD_E_NOMEM: return "out of device memory or budget";
    case RD_E_DEVICE: return "HIP runtime error";
    case RD_E_BUSY: return "not finished";
    }
    return "unknown status";
}

void rd_default_opts(rd_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->max_iter = 10000;
    o->max_outer = 20;
    o->tau_u = 0.9;
    o->tau_p = 0.9;
    o->omega = 1.0;
    o->precision = RD_FP64;
    o->init = RD_INIT_PREV;
    o->inner_rtol = 3e-2;
}

rd_status rd_create(int device, rd_ctx **out) {
    if (!out) return RD_E_INVALID;
    *out = nullptr;
    int n = 0;
    RD_CHECK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return RD_E_INVALID;
    RD_CHECK(hipSetDevice(device));
    std::call_once(g_register_once, register_all);
    rd_status r = noalloc_setup(device);
    if (r != RD_OK) return r;
    auto *c = new Ctx();
    c->device = device;
    if (hipMalloc((void **)&c->scratch_slot_dev, sizeof(Slot)) != hipSuccess ||
        hipHostMalloc((void **)&c->scratch_slot_host, sizeof(Slot), hipHostMallocDefault) != hipSuccess) {
        if (c->scratch_slot_dev) (void)hipFree(c->scratch_slot_dev);
        delete c;
        return RD_E_NOMEM;
    }
    *out = (rd_ctx *)c;
    return RD_OK;
}

rd_status rd_destroy(rd_ctx *ctx) {
    if (!ctx) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (Traj *t : c->trajs) {
        if (t->ws) free_workspace(t->ws.get());
        if (t->u) (void)hipFree(t->u);
        delete t;
    }
    for (auto &kv : c->step_ws) free_workspace(kv.second.get());
    for (auto &kv : c->tables) {
        (void)hipFree(kv.second.eig);
        for (int i = 0; i < 2; ++i) {
            (void)hipFree(kv.second.tw[i]);
            (void)hipFree(kv.second.twd[i]);
        }
    }
    for (auto &kv : c->rounds) {
        if (kv.second.stream) (void)hipStreamDestroy(kv.second.stream);
        if (kv.second.done) (void)hipEventDestroy(kv.second.done);
    }
    for (auto &kv : c->batch) {
        if (kv.second.dev) (void)hipFree(kv.second.dev);
        if (kv.second.host) (void)hipHostFree(kv.second.host);
    }
    if (c->scratch_slot_dev) (void)hipFree(c->scratch_slot_dev);
    if (c->scratch_slot_host) (void)hipHostFree(c->scratch_slot_host);
    if (c->scratch_partials) (void)hipFree(c->scratch_partials);
    delete c;
    return RD_OK;
}

size_t rd_footprint_bytes(const rd_problem *prob, const rd_opts *opts) {
    Desc d;
    if (describe(prob, d) != RD_OK || check_opts(opts) != RD_OK) return 0;
    std::call_once(g_register_once, register_all);
    const int mode = opts->precision == RD_FP32_MIXED ? MODE_MIXED : MODE_F64;
    if (!kset(mode, d).init) return 0;   // no such precision for the equation
    const int rpb = kset(mode, d).rows_per_block;
    // resident trajectory state + the step workspace
    return workspace_bytes(d.pts, d.rows, d.C, mode, rpb) + field_bytes(d.pts, d.C, 8);
}

rd_status rd_step(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts, double h_t, const double *u_n,
                  double *u_np1, void *hip_stream, rd_info *info) {
    if (!ctx || !u_n || !u_np1) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    Desc d;
    rd_status r = describe(prob, d);
    if (r != RD_OK) return r;
    if ((r = check_opts(opts)) != RD_OK) return r;
    if (!(h_t > 0.0) || !std::isfinite(h_t)) return RD_E_INVALID;
    RD_CHECK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const int mode = opts->precision == RD_FP32_MIXED ? MODE_MIXED : MODE_F64;
    const KSet &k = kset(mode, d);
    if (!k.init) return RD_E_INVALID;   // no such precision for the equation
    Tables *t = nullptr;
    if ((r = get_tables(c, d.N, d.bc, d.h, t)) != RD_OK) return r;
    Workspace *w = nullptr;
    if ((r = get_step_workspace(c, d, mode, w)) != RD_OK) return r;
    Slot &s = *w->slot_host;
    std::memset(&s, 0, sizeof(Slot));
    fill_params(s, prob, opts, d, h_t);
    bind_workspace(s, *w, *t);
    s.src = u_n;
    const size_t n = (size_t)d.C * d.pts;
    const bool dev_copy = ((uintptr_t)u_np1 % 32) == 0 && n % 4 == 0;
    // The output serves as the FP64 iterate buffer the previous step ended in (that
    // index is as steady as the step's length), so a step that ends there needs no
    // copy.  Buffer 0 is written by the initial pass while it reads u_n, so it is
    // taken only when the output does not overlap u_n.
    if (dev_copy && w->last_parity >= 0) {
        const int p = w->last_parity;
        const char *a = (const char *)u_np1, *b = (const char *)u_n;
        const size_t bytes = n * sizeof(double);
        if (p == 1 || !(a < b + bytes && b < a + bytes)) {
            if (mode == MODE_F64) s.U[p] = u_np1;
            else s.U64[p] = u_np1;
        }
    }
    RD_CHECK(hipMemcpyAsync(w->slot_dev, &s, sizeof(Slot), hipMemcpyHostToDevice, st));
    if ((r = run_step(c, *w, k, st, opts->max_iter, opts->max_outer, dev_copy ? u_np1 : nullptr, n)) != RD_OK)
        return r;
    const State &sf = *w->st_host;
    if (!dev_copy) {
        RD_CHECK(hipMemcpyAsync(u_np1, final_buffer(*w, sf), field_bytes(d.pts, d.C, 8), hipMemcpyDeviceToDevice,
                                st));
        RD_CHECK(hipStreamSynchronize(st));
    }
    info_from_state(sf, mode, info);
    return (rd_status)sf.status;
}

rd_status rd_step_noalloc(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts, double h_t, const double *u_n,
                          double *u_np1, void *hip_stream, rd_info *info) {
    if (!ctx || !u_n || !u_np1) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    Desc d;
    rd_status r = describe(prob, d);
    if (r != RD_OK) return r;
    if ((r = check_opts(opts)) != RD_OK) return r;
    if (!(h_t > 0.0) || !std::isfinite(h_t)) return RD_E_INVALID;
    const int mode = opts->precision == RD_FP32_MIXED ? MODE_MIXED : MODE_F64;
    const KSet &k = kset(mode, d);
    if (!k.init) return RD_E_INVALID;   // no such precision for the equation
    if (c->device >= NOALLOC_MAX_DEVICES || !g_noalloc[c->device].base) return RD_E_DEVICE;
    if (d.N > NOALLOC_MAX_N) return RD_E_NOMEM;
    NoAllocDevice &na = g_noalloc[c->device];
    RD_CHECK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    // the workspace of rd_step, carved from the scratch array (256-byte aligned pieces)
    const int C = d.C;
    const size_t te = mode == MODE_F64 ? 8 : 4;
    const int nblk = d.rows / k.rows_per_block;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t o_slot = take(sizeof(Slot)), o_list = take(sizeof(Slot *)), o_st = take(sizeof(State));
    const size_t o_part = take((size_t)nblk * 2 * C * sizeof(double));
    const size_t o_eig = take((size_t)d.N * sizeof(double));
    const size_t o_tw = take(2 * (size_t)d.N * te), o_twd = take(2 * (size_t)d.N * te);
    const size_t fb = field_bytes(d.pts, C, te), f64 = field_bytes(d.pts, C, 8), f32 = field_bytes(d.pts, C, 4);
    const size_t o_u0 = take(fb), o_u1 = take(fb), o_p = take(fb), o_pt = take(fb), o_s = take(fb);
    const size_t o_uk = take(f64);
    size_t o_v0 = 0, o_v1 = 0, o_r = 0, o_ub = 0;
    if (mode == MODE_MIXED) {
        o_v0 = take(f64);
        o_v1 = take(f64);
        o_r = take(f32);
        o_ub = take(f32);
    }
    if (off > NOALLOC_BYTES) return RD_E_NOMEM;
    char *B = na.base;
    // tables, in the iteration's precision
    fill_tables_host(d.N, d.bc, d.h, na.eig, na.tw, na.twd);
    RD_CHECK(hipMemcpyAsync(B + o_eig, na.eig, (size_t)d.N * sizeof(double), hipMemcpyHostToDevice, st));
    if (mode == MODE_F64) {
        RD_CHECK(hipMemcpyAsync(B + o_tw, na.tw, 2 * (size_t)d.N * sizeof(double), hipMemcpyHostToDevice, st));
        RD_CHECK(hipMemcpyAsync(B + o_twd, na.twd, 2 * (size_t)d.N * sizeof(double), hipMemcpyHostToDevice, st));
    } else {
        for (int i = 0; i < 2 * d.N; ++i) {
            na.tw32[i] = (float)na.tw[i];
            na.twd32[i] = (float)na.twd[i];
        }
        RD_CHECK(hipMemcpyAsync(B + o_tw, na.tw32, 2 * (size_t)d.N * sizeof(float), hipMemcpyHostToDevice, st));
        RD_CHECK(hipMemcpyAsync(B + o_twd, na.twd32, 2 * (size_t)d.N * sizeof(float), hipMemcpyHostToDevice, st));
    }
    // the slot, its one-entry list and a zeroed State
    Slot &s = na.slot;
    std::memset(&s, 0, sizeof(Slot));
    fill_params(s, prob, opts, d, h_t);
    s.U[0] = B + o_u0;
    s.U[1] = B + o_u1;
    s.P = B + o_p;
    s.Pt = B + o_pt;
    s.S = B + o_s;
    s.Uk = (double *)(B + o_uk);
    if (mode == MODE_MIXED) {
        s.U64[0] = (double *)(B + o_v0);
        s.U64[1] = (double *)(B + o_v1);
        s.r32 = (float *)(B + o_r);
        s.Ub32 = (float *)(B + o_ub);
    }
    s.partials = (double *)(B + o_part);
    s.st = (State *)(B + o_st);
    s.nblk_rows = nblk;
    s.eig = (const double *)(B + o_eig);
    s.tw = B + o_tw;
    s.twd = B + o_twd;
    s.src = u_n;
    na.list = (Slot *)(B + o_slot);
    std::memset(&na.st, 0, sizeof(State));
    RD_CHECK(hipMemcpyAsync(B + o_slot, &s, sizeof(Slot), hipMemcpyHostToDevice, st));
    RD_CHECK(hipMemcpyAsync(B + o_list, &na.list, sizeof(Slot *), hipMemcpyHostToDevice, st));
    RD_CHECK(hipMemcpyAsync(B + o_st, &na.st, sizeof(State), hipMemcpyHostToDevice, st));
    // the launch schedule of rd_step on a workspace that owns nothing
    Workspace w;
    w.N = d.N;
    w.C = C;
    w.mode = mode;
    w.logN = d.logN;
    w.nblk = nblk;
    w.dim = d.dim;
    w.pts = d.pts;
    w.proto = s;
    w.slot_dev = (Slot *)(B + o_slot);
    w.slot_list_dev = (Slot **)(B + o_list);
    w.st_host = &na.st;
    w.last_iters = na.last_iters;
    w.prev_iters = na.prev_iters;
    const size_t n = (size_t)C * d.pts;
    const bool dev_copy = ((uintptr_t)u_np1 % 32) == 0 && n % 4 == 0;
    r = run_step(c, w, k, st, opts->max_iter, opts->max_outer, dev_copy ? u_np1 : nullptr, n);
    na.last_iters = w.last_iters;
    na.prev_iters = w.prev_iters;
    if (r != RD_OK) return r;
    const State &sf = na.st;
    if (!dev_copy) {
        RD_CHECK(hipMemcpyAsync(u_np1, final_buffer(w, sf), field_bytes(d.pts, C, 8), hipMemcpyDeviceToDevice, st));
        RD_CHECK(hipStreamSynchronize(st));
    }
    info_from_state(sf, mode, info);
    return (rd_status)sf.status;
}

rd_status rd_profile_iteration(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts, double h_t,
                               const double *u_n, int32_t reps, void *hip_stream, double *ms_out) {
    if (!ctx || !u_n || !ms_out || reps <= 0) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    Desc d;
    rd_status r = describe(prob, d);
    if (r != RD_OK) return r;
    if ((r = check_opts(opts)) != RD_OK) return r;
    if (!(h_t > 0.0)) return RD_E_INVALID;
    RD_CHECK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const int mode = opts->precision == RD_FP32_MIXED ? MODE_MIXED : MODE_F64;
    const KSet &k = kset(mode, d);
    if (!k.init) return RD_E_INVALID;   // no such precision for the equation
    Tables *t = nullptr;
    if ((r = get_tables(c, d.N, d.bc, d.h, t)) != RD_OK) return r;
    Workspace *w = nullptr;
    if ((r = get_step_workspace(c, d, mode, w)) != RD_OK) return r;
    Slot &s = *w->slot_host;
    std::memset(&s, 0, sizeof(Slot));
    fill_params(s, prob, opts, d, h_t);
    bind_workspace(s, *w, *t);
    s.src = u_n;
    s.max_iter = 1 << 30;   // the stop decision must not end the timed launches
    s.tol = 0.0;
    RD_CHECK(hipMemcpyAsync(w->slot_dev, &s, sizeof(Slot), hipMemcpyHostToDevice, st));
    k.init(w->slot_list_dev, 1, st, nullptr);
    // The solver's launch order of one iteration (the stop decision of a row pass is
    // taken by the next column pass, 2-D, or forward y pass, 3-D).
    std::vector<launch_fn> fns;
    if (d.dim == 3)
        fns = {k.yfwd_fin, k.zsym, k.yinv, k.rowinv, k.upd, k.rowfwd};
    else
        fns = {k.cols_fin, k.rowinv, k.upd, k.rowfwd};
    const int nk = (int)fns.size();
    // One untimed iteration from the initial state (whose decision the initial
    // pass has taken).
    for (int kk = 0; kk < nk; ++kk)
        (kk == 0 ? (d.dim == 3 ? k.yfwd : k.cols) : fns[kk])(w->slot_list_dev, 1, st, nullptr);
    RD_CHECK(hipGetLastError());
    RD_CHECK(hipStreamSynchronize(st));
    // No stop rule may end the timed iterations: tolerance 0 and max_iter 2^30 are
    // in the slot; the mixed inner loop's target and stall rule are disabled here.
    State run{};
    RD_CHECK(hipMemcpy(&run, w->proto.st, sizeof(State), hipMemcpyDeviceToHost));
    if (run.status != ST_OK) return RD_E_NONFINITE;
    run.done = 0;
    run.outer_done = 0;
    run.inner_target = 0.0;
    run.inner_best = 0.0;
    run.inner_best_it = 1 << 29;
    if (run.res0 == 0.0) run.res0 = 1.0;
    *w->st_host = run;
    RD_CHECK(hipMemcpyAsync(w->proto.st, w->st_host, sizeof(State), hipMemcpyHostToDevice, st));
    // reps iterations in the solver's launch order, back to back; every launch's
    // dispatch packets record a start and a stop event (the kernel's own begin and
    // end), so each kernel is timed in the cache state the real loop leaves it.
    std::vector<hipEvent_t> ev(2 * (size_t)nk * reps);
    for (auto &e : ev) RD_CHECK(hipEventCreate(&e));
    for (int i = 0; i < reps; ++i)
        for (int kk = 0; kk < nk; ++kk) fns[kk](w->slot_list_dev, 1, st, &ev[2 * (nk * i + kk)]);
    RD_CHECK(hipGetLastError());
    RD_CHECK(hipStreamSynchronize(st));
    for (int kk = 0; kk < nk; ++kk) {
        double tot = 0.0;
        for (int i = 0; i < reps; ++i) {
            float ms = 0.f;
            RD_CHECK(hipEventElapsedTime(&ms, ev[2 * (nk * i + kk)], ev[2 * (nk * i + kk) + 1]));
            tot += ms;
        }
        ms_out[kk] = tot / reps;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return RD_OK;
}

// ---------------------------------------------------------------- adaptive time step size
}  // extern "C"

namespace {
bool check_adapt(const rd_adapt *a) {
    return a && a->ht0 > 0.0 && std::isfinite(a->ht0) && a->eta > 0.0 && a->eta < 1.0 && a->n_lo > 0 &&
           a->n_hi > a->n_lo && a->ht_min >= 0.0 && a->max_rejects >= 0;
}
bool reached(double t, double t_end) { return t_end - t <= 1e-14 * std::max(1.0, std::fabs(t_end)); }
}  // namespace

extern "C" {

rd_status rd_adapt_next(const rd_adapt *a, double h, int32_t iters, int32_t step_status, double *ht_next,
                        int32_t *accept) {
    if (!check_adapt(a) || !ht_next || !accept || !(h > 0.0)) return RD_E_INVALID;
    if (step_status != RD_OK) {
        *ht_next = a->eta * h;
        *accept = 0;
        return RD_OK;
    }
    *accept = 1;
    if (iters > a->n_hi) {
        *ht_next = a->eta * h;
    } else if (iters < a->n_lo) {
        const double up = h / a->eta;
        *ht_next = up <= a->ht0 ? up : h;
    } else {
        *ht_next = h;
    }
    return RD_OK;
}

rd_status rd_advance(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts, const rd_adapt *a, double t0,
                     double t_end, double *u, void *hip_stream, rd_adapt_info *info, double *trace_h,
                     int32_t *trace_iters, int32_t *trace_ok, int32_t trace_cap) {
    if (!ctx || !u || !info || !check_adapt(a) || !std::isfinite(t0) || !std::isfinite(t_end) || t_end < t0)
        return RD_E_INVALID;
    if (trace_cap < 0 || (trace_cap > 0 && (!trace_h || !trace_iters || !trace_ok))) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    Desc d;
    rd_status r = describe(prob, d);
    if (r != RD_OK) return r;
    if ((r = check_opts(opts)) != RD_OK) return r;
    RD_CHECK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t fb = field_bytes(d.pts, d.C, 8);
    double *next = nullptr;
    if (hipMalloc((void **)&next, fb) != hipSuccess) return RD_E_NOMEM;
    std::memset(info, 0, sizeof(*info));
    double t = t0, ht = a->ht0;
    int rejects = 0, n = 0;
    rd_status out = RD_OK;
    while (!reached(t, t_end)) {
        const double h = std::min(ht, t_end - t);
        rd_info si;
        r = rd_step(ctx, prob, opts, h, u, next, hip_stream, &si);
        if (r == RD_E_INVALID || r == RD_E_DEVICE || r == RD_E_NOMEM) {
            out = r;
            break;
        }
        info->pdhg_iters += si.iters;
        double nxt = h;
        int32_t ok = 0;
        rd_adapt_next(a, h, si.iters, si.status, &nxt, &ok);
        if (n < trace_cap) {
            trace_h[n] = h;
            trace_iters[n] = si.iters;
            trace_ok[n] = ok;
        }
        ++n;
        if (ok) {
            if (hipMemcpyAsync(u, next, fb, hipMemcpyDeviceToDevice, st) != hipSuccess) {
                out = RD_E_DEVICE;
                break;
            }
            t = t + h;
            ++info->accepted;
            rejects = 0;
        } else {
            ++info->rejected;
            ++rejects;
        }
        if (nxt < h) ++info->shrinks;
        else if (nxt > h) ++info->enlarges;
        ht = nxt;
        if (!ok && (ht < a->ht_min || rejects > a->max_rejects)) {
            out = RD_E_NOCONV;
            break;
        }
    }
    const bool synced = hipStreamSynchronize(st) == hipSuccess;
    (void)hipFree(next);
    if (!synced && out == RD_OK) out = RD_E_DEVICE;
    info->t = t;
    info->ht = ht;
    info->status = out;
    return out;
}

// ---------------------------------------------------------------- kernel-level entry points
rd_status rd_residual(rd_ctx *ctx, const rd_problem *prob, double h_t, const double *u, const double *uk, double *w,
                      void *hip_stream, double *res_l2) {
    if (!ctx || !u || !uk || !w) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    Desc d;
    rd_status r = describe(prob, d);
    if (r != RD_OK) return r;
    if (!(h_t > 0.0) || d.dim != 2) return RD_E_INVALID;   // kernel-level calls: 2-D grids
    RD_CHECK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    Slot &s = *c->scratch_slot_host;
    std::memset(&s, 0, sizeof(Slot));
    fill_params(s, prob, nullptr, d, h_t);
    const size_t blocks = ((size_t)d.N * d.N + NT - 1) / NT;
    const size_t need = blocks * d.C;
    if (c->scratch_partials_n < need) {
        if (c->scratch_partials) (void)hipFree(c->scratch_partials);
        c->scratch_partials = nullptr;
        c->scratch_partials_n = 0;
        RD_CHECK(hipMalloc((void **)&c->scratch_partials, need * sizeof(double)));
        c->scratch_partials_n = need;
    }
    RD_CHECK(hipMemcpyAsync(c->scratch_slot_dev, &s, sizeof(Slot), hipMemcpyHostToDevice, st));
    launch_residual(d.bc, d.eq, c->scratch_slot_dev, d.N, u, uk, w, c->scratch_partials, st);
    RD_CHECK(hipGetLastError());
    c->host_partials.resize(need);
    RD_CHECK(hipMemcpyAsync(c->host_partials.data(), c->scratch_partials, need * sizeof(double),
                            hipMemcpyDeviceToHost, st));
    RD_CHECK(hipStreamSynchronize(st));
    if (res_l2) {
        double res = 0.0;
        for (int comp = 0; comp < d.C; ++comp) {
            double acc = 0.0;
            for (size_t b = 0; b < blocks; ++b) acc += c->host_partials[b * d.C + comp];
            res += std::sqrt(acc);
        }
        *res_l2 = res / h_t;
    }
    return RD_OK;
}

rd_status rd_precond_solve(rd_ctx *ctx, const rd_problem *prob, double h_t, int32_t precision, const double *w_in,
                           double *y, void *hip_stream) {
    if (!ctx || !w_in || !y) return RD_E_INVALID;
    if (precision != RD_FP64 && precision != RD_FP32_MIXED) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    Desc d;
    rd_status r = describe(prob, d);
    if (r != RD_OK) return r;
    if (!(h_t > 0.0)) return RD_E_INVALID;
    RD_CHECK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const int mode = precision == RD_FP32_MIXED ? MODE_MIXED : MODE_F64;
    const KSet &k = kset(mode, d);
    if (!k.tin) return RD_E_INVALID;   // no such precision for the equation
    Tables *t = nullptr;
    if ((r = get_tables(c, d.N, d.bc, d.h, t)) != RD_OK) return r;
    Workspace *w = nullptr;
    if ((r = get_step_workspace(c, d, mode, w)) != RD_OK) return r;
    Slot &s = *w->slot_host;
    std::memset(&s, 0, sizeof(Slot));
    fill_params(s, prob, nullptr, d, h_t);
    bind_workspace(s, *w, *t);
    RD_CHECK(hipMemcpyAsync(w->slot_dev, &s, sizeof(Slot), hipMemcpyHostToDevice, st));
    RD_CHECK(hipMemsetAsync(w->proto.st, 0, sizeof(State), st));   // unfinished State: the passes run
    k.tin(w->slot_list_dev, 1, w_in, nullptr, st);
    if (d.dim == 3) {
        k.yfwd(w->slot_list_dev, 1, st, nullptr);
        k.zsym(w->slot_list_dev, 1, st, nullptr);
        k.yinv(w->slot_list_dev, 1, st, nullptr);
    } else {
        k.cols(w->slot_list_dev, 1, st, nullptr);
    }
    k.tout(w->slot_list_dev, 1, nullptr, y, st);
    RD_CHECK(hipGetLastError());
    RD_CHECK(hipStreamSynchronize(st));
    return RD_OK;
}

rd_status rd_prox(rd_ctx *ctx, const rd_problem *prob, double h_t, const double *cin, double *u, void *hip_stream) {
    if (!ctx || !cin || !u) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    Desc d;
    rd_status r = describe(prob, d);
    if (r != RD_OK) return r;
    if (!(h_t > 0.0) || d.dim != 2) return RD_E_INVALID;   // kernel-level calls: 2-D grids
    RD_CHECK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    Slot &s = *c->scratch_slot_host;
    std::memset(&s, 0, sizeof(Slot));
    fill_params(s, prob, nullptr, d, h_t);
    RD_CHECK(hipMemcpyAsync(c->scratch_slot_dev, &s, sizeof(Slot), hipMemcpyHostToDevice, st));
    launch_prox(d.eq, c->scratch_slot_dev, d.N, cin, u, st);
    RD_CHECK(hipGetLastError());
    RD_CHECK(hipStreamSynchronize(st));
    return RD_OK;
}

// ---------------------------------------------------------------- serving
rd_status rd_serve_set_budget(rd_ctx *ctx, size_t bytes) {
    if (!ctx) return RD_E_INVALID;
    ((Ctx *)ctx)->budget = bytes;
    return RD_OK;
}

rd_status rd_traj_open(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts, const double *u0, void *hip_stream,
                       rd_traj **out) {
    if (!ctx || !u0 || !out) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    Desc d;
    rd_status r = describe(prob, d);
    if (r != RD_OK) return r;
    if ((r = check_opts(opts)) != RD_OK) return r;
    RD_CHECK(hipSetDevice(c->device));
    auto *t = new Traj();
    t->ctx = c;
    t->prob = *prob;
    t->opts = *opts;
    t->d = d;
    t->d.mode = opts->precision == RD_FP32_MIXED ? MODE_MIXED : MODE_F64;
    if (!kset(t->d.mode, t->d).init) {   // no such precision for the equation
        delete t;
        return RD_E_INVALID;
    }
    const size_t fb = field_bytes(d.pts, d.C, 8);
    if (hipMalloc((void **)&t->u, fb) != hipSuccess) {
        delete t;
        return RD_E_NOMEM;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if (hipMemcpyAsync(t->u, u0, fb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipFree(t->u);
        delete t;
        return RD_E_DEVICE;
    }
    c->trajs.push_back(t);
    *out = (rd_traj *)t;
    return RD_OK;
}

rd_status rd_traj_submit(rd_traj *traj, double h_t, uint64_t *ticket) {
    if (!traj || !ticket || !(h_t > 0.0) || !std::isfinite(h_t)) return RD_E_INVALID;
    Traj *t = (Traj *)traj;
    Ctx *c = t->ctx;
    const uint64_t id = c->next_ticket++;
    c->tickets[id] = Ticket{};
    t->tickets.push_back(id);
    t->pending.push_back(PendingStep{id, h_t});
    if (!t->ws && !t->queued_for_admission) {
        c->admit_queue.push_back(t);
        t->queued_for_admission = true;
    }
    *ticket = id;
    return RD_OK;
}

}  // extern "C"

namespace {

// Serving.  A pump call:
//  1. admits queued trajectories in arrival order while the resident budget allows;
//  2. retires the rounds that have completed: finished steps' tickets get their
//     info (the results were already copied into the resident states on the
//     device);
//  3. starts a round for every group with work and no round in flight: the next
//     pending step of each idle admitted trajectory (batched initial pass), and
//     one chunk of iterations for all running slots of the group (one launch per
//     kernel; small grids run their whole steps in one launch);
//  4. if no round had completed, waits for the first one that does (at most
//     max_wait_us when that is > 0), retires it and restarts its group.
// Groups run on their own streams and finish independently: a short step is not
// held behind the iterations of another group's long one.

rd_status batch_list(Ctx *c, const GroupKey &key, int role, const std::vector<Traj *> &ts, Slot **&dev,
                     hipStream_t st) {
    BatchBuffers &b = c->batch[std::make_pair(key, role)];
    const int n = (int)ts.size();
    if (b.cap < n) {
        if (b.dev) (void)hipFree(b.dev);
        if (b.host) (void)hipHostFree(b.host);
        b.dev = nullptr;
        b.host = nullptr;
        b.cap = 0;
        const int cap = std::max(16, 2 * n);
        RD_CHECK(hipMalloc((void **)&b.dev, cap * sizeof(Slot *)));
        RD_CHECK(hipHostMalloc((void **)&b.host, cap * sizeof(Slot *), hipHostMallocDefault));
        b.cap = cap;
    }
    for (int i = 0; i < n; ++i) b.host[i] = ts[i]->ws->slot_dev;
    RD_CHECK(hipMemcpyAsync(b.dev, b.host, n * sizeof(Slot *), hipMemcpyHostToDevice, st));
    dev = b.dev;
    return RD_OK;
}

// Retire a completed round: record the finished steps' tickets.
void retire_round(Ctx *c, GroupRound &g) {
    for (Traj *t : g.trajs) {
        Workspace &w = *t->ws;
        const State &s = *w.st_host;
        const bool fin = w.mode == MODE_F64 ? s.done != 0 : s.outer_done != 0;
        if (!fin) continue;
        Ticket &tk = c->tickets[t->running_ticket];
        info_from_state(s, w.mode, &tk.info);
        tk.done = true;
        remember_step(w, s);
        t->running = false;
    }
    g.trajs.clear();
    g.in_flight = false;
}

// Retire every in-flight round whose work has completed; retired counts them.
rd_status poll_rounds(Ctx *c, int &retired) {
    retired = 0;
    for (auto &kv : c->rounds) {
        GroupRound &g = kv.second;
        if (!g.in_flight) continue;
        const hipError_t e = hipEventQuery(g.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return RD_E_DEVICE;
        retire_round(c, g);
        ++retired;
    }
    return RD_OK;
}

// Start a round for every batch group that has work and no round in flight.
rd_status launch_rounds(Ctx *c) {
    rd_status r;
    std::map<GroupKey, std::vector<Traj *>> starting, running;
    for (Traj *t : c->trajs) {
        if (!t->ws) continue;
        GroupKey key{t->d.mode, t->d.logN, t->d.bc, t->d.eq, t->d.dim};
        auto gi = c->rounds.find(key);
        if (gi != c->rounds.end() && gi->second.in_flight) continue;
        if (!t->running && !t->pending.empty()) {
            starting[key].push_back(t);
            running[key].push_back(t);
        } else if (t->running) {
            running[key].push_back(t);
        }
    }
    for (auto &kv : running) {
        const GroupKey &key = kv.first;
        GroupRound &g = c->rounds[key];
        if (!g.stream) RD_CHECK(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
        if (!g.done) RD_CHECK(hipEventCreateWithFlags(&g.done, hipEventDisableTiming));
        hipStream_t st = g.stream;
        const KSet &k = kset(key.mode, kv.second.front()->d);
        const size_t nfield = (size_t)kv.second.front()->d.C * kv.second.front()->d.pts;
        auto si = starting.find(key);
        if (si != starting.end()) {
            for (Traj *t : si->second) {
                PendingStep ps = t->pending.front();
                t->pending.pop_front();
                Tables *tb = nullptr;
                if ((r = get_tables(c, t->d.N, t->d.bc, t->d.h, tb)) != RD_OK) return r;
                Slot &s = *t->ws->slot_host;
                std::memset(&s, 0, sizeof(Slot));
                fill_params(s, &t->prob, &t->opts, t->d, ps.ht);
                bind_workspace(s, *t->ws, *tb);
                s.src = t->u;
                RD_CHECK(hipMemcpyAsync(t->ws->slot_dev, &s, sizeof(Slot), hipMemcpyHostToDevice, st));
                t->running = true;
                t->running_ticket = ps.ticket;
                t->issued = 0;
            }
            Slot **dev = nullptr;
            if ((r = batch_list(c, key, 0, si->second, dev, st)) != RD_OK) return r;
            if (k.step_wg) {
                // small grids: the whole steps in one launch, one workgroup each
                const int n = (int)si->second.size();
                k.step_wg(dev, n, st, nullptr);
                launch_copy_back(dev, n, nfield, st);
            } else {
                k.init(dev, (int)si->second.size(), st, nullptr);
            }
            RD_CHECK(hipGetLastError());
        }
        if (!k.step_wg) {
            Slot **dev = nullptr;
            if ((r = batch_list(c, key, 1, kv.second, dev, st)) != RD_OK) return r;
            // Chunk length: the trajectory's previous step predicts this one; a step
            // that runs longer grows its chunks geometrically (fewer host round
            // trips), up to 32 iterations, so that a group's completion is seen soon
            // enough to start its next steps.
            int iters = 0;
            for (Traj *t : kv.second) {
                const Workspace &w = *t->ws;
                iters = std::max(iters, std::max(first_chunk(w), t->issued / 2));
            }
            iters = std::min(iters, 32);
            for (Traj *t : kv.second) t->issued += iters;
            enqueue_round(k, dev, (int)kv.second.size(), iters, st);
            // steps that finish in this round: U^{k+1} becomes the resident state on
            // the device, before the host has looked at any State
            launch_copy_back(dev, (int)kv.second.size(), nfield, st);
            RD_CHECK(hipGetLastError());
        }
        for (Traj *t : kv.second)
            RD_CHECK(hipMemcpyAsync(t->ws->st_host, t->ws->proto.st, sizeof(State), hipMemcpyDeviceToHost, st));
        RD_CHECK(hipEventRecord(g.done, st));
        g.trajs = kv.second;
        g.in_flight = true;
    }
    return RD_OK;
}

}  // namespace

extern "C" {

rd_status rd_serve_pump(rd_ctx *ctx, int32_t max_wait_us) {
    if (!ctx || max_wait_us < 0) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    RD_CHECK(hipSetDevice(c->device));
    rd_status r;
    // 1. admission, in arrival order, while the resident budget allows
    while (!c->admit_queue.empty()) {
        Traj *t = c->admit_queue.front();
        const size_t need = workspace_bytes(t->d.pts, t->d.rows, t->d.C, t->d.mode,
                                            kset(t->d.mode, t->d).rows_per_block);
        if (c->budget && c->resident + need > c->budget && c->resident > 0) break;
        std::unique_ptr<Workspace> w;
        r = make_workspace(t->d, t->d.mode, w);
        if (r == RD_E_NOMEM && c->resident > 0) break;
        if (r != RD_OK) return r;
        t->ws = std::move(w);
        c->resident += need;
        c->admit_queue.pop_front();
        t->queued_for_admission = false;
    }
    // 2. retire completed rounds, 3. start rounds for idle groups
    int retired = 0;
    if ((r = poll_rounds(c, retired)) != RD_OK) return r;
    if ((r = launch_rounds(c)) != RD_OK) return r;
    // 4. wait for the first completion, then restart that group
    if (retired == 0) {
        bool any = false;
        for (auto &kv : c->rounds) any = any || kv.second.in_flight;
        if (any) {
            const auto t0 = std::chrono::steady_clock::now();
            while (true) {
                if ((r = poll_rounds(c, retired)) != RD_OK) return r;
                if (retired > 0) break;
                if (max_wait_us > 0 && std::chrono::duration_cast<std::chrono::microseconds>(
                                           std::chrono::steady_clock::now() - t0).count() >= max_wait_us)
                    break;
                std::this_thread::yield();
            }
            if (retired > 0 && (r = launch_rounds(c)) != RD_OK) return r;
        }
    }
    return RD_OK;
}

rd_status rd_serve_stats(rd_ctx *ctx, rd_serve_info *out) {
    if (!ctx || !out) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    std::memset(out, 0, sizeof(*out));
    out->budget_bytes = c->budget;
    out->resident_bytes = c->resident;
    for (Traj *t : c->trajs) {
        if (t->ws) ++out->admitted;
        if (t->running) ++out->running;
        out->pending_steps += (int32_t)t->pending.size();
    }
    out->queued = (int32_t)c->admit_queue.size();
    return RD_OK;
}

rd_status rd_poll(rd_ctx *ctx, uint64_t ticket, rd_info *info) {
    if (!ctx) return RD_E_INVALID;
    Ctx *c = (Ctx *)ctx;
    auto it = c->tickets.find(ticket);
    if (it == c->tickets.end()) return RD_E_INVALID;
    if (!it->second.done) return RD_E_BUSY;
    if (info) *info = it->second.info;
    return (rd_status)it->second.info.status;
}

rd_status rd_traj_read(rd_traj *traj, double *u_out, void *hip_stream) {
    if (!traj || !u_out) return RD_E_INVALID;
    Traj *t = (Traj *)traj;
    RD_CHECK(hipSetDevice(t->ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    // a round in flight that advances t replaces its resident state when a step
    // finishes: the copy waits for that round, so it never sees a state half written
    for (auto &kv : t->ctx->rounds) {
        const GroupRound &g = kv.second;
        if (g.in_flight && std::find(g.trajs.begin(), g.trajs.end(), t) != g.trajs.end())
            RD_CHECK(hipStreamWaitEvent(st, g.done, 0));
    }
    RD_CHECK(hipMemcpyAsync(u_out, t->u, field_bytes(t->d.pts, t->d.C, 8), hipMemcpyDeviceToDevice, st));
    RD_CHECK(hipStreamSynchronize(st));
    return RD_OK;
}

rd_status rd_traj_close(rd_traj *traj) {
    if (!traj) return RD_E_INVALID;
    Traj *t = (Traj *)traj;
    Ctx *c = t->ctx;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    // every round has completed: retire them, so that none refers to t afterwards
    for (auto &kv : c->rounds)
        if (kv.second.in_flight) retire_round(c, kv.second);
    if (t->ws) {
        c->resident -= std::min(c->resident, t->ws->bytes);
        free_workspace(t->ws.get());
        t->ws.reset();
    }
    for (size_t i = 0; i < c->admit_queue.size(); ++i)
        if (c->admit_queue[i] == t) {
            c->admit_queue.erase(c->admit_queue.begin() + i);
            break;
        }
    for (size_t i = 0; i < c->trajs.size(); ++i)
        if (c->trajs[i] == t) {
            c->trajs.erase(c->trajs.begin() + i);
            break;
        }
    // its tickets, finished or not, become unknown: no poll waits on a step that will
    // never run, and the ticket table holds the open trajectories' steps only
    for (uint64_t id : t->tickets) c->tickets.erase(id);
    if (t->u) (void)hipFree(t->u);
    delete t;
    return RD_OK;
}

}  // extern "C"
