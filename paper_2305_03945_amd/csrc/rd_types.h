// Plain data of the device path, shared by the HIP kernels and the host runtime
// and compilable as ordinary C++ (the host-only checks build the runtime against
// a stub of the HIP API): equation and precision codes, the per-slot parameters
// and iteration state, and the stop decision taken after each residual pass.
#pragma once
#include <math.h>
#include <stdint.h>

#if defined(__HIP__)
#define RD_HD __host__ __device__
#else
#define RD_HD
#endif

namespace rdk {

// Equation family: fixes the stencil shape and the number of components.
//   EQ_LAP5   : +lambda Lap (5-point) with the Allen-Cahn reaction (b = 0: heat)
//   EQ_BIH    : -lambda Lap Lap (13-point) with + Lap g(u) (b = 0: biharmonic)
//   EQ_SCHNAK : two components, 5-point Laplacians, Schnakenberg kinetics
//   EQ_FCH    : sixth-order functionalized Cahn-Hilliard (nested 5-point Laplacians,
//               25-point reach), FP64 only
enum { EQ_LAP5 = 0, EQ_BIH = 1, EQ_SCHNAK = 2, EQ_FCH = 3, EQ_COUNT = 4 };
enum { BC_P = 0, BC_N = 1 };
// Precision mode of a step: plain FP64 iteration, or FP32 inner iteration on a
// correction with FP64 outer residual passes.
enum { MODE_F64 = 0, MODE_MIXED = 1 };

// Step status codes (same values as rd_status).
enum { ST_OK = 0, ST_NOCONV = -2, ST_NONFINITE = -3 };

constexpr int NT = 256;                 // threads per workgroup, every kernel
constexpr double GROWTH_LIMIT = 1e8;    // residual growth that counts as divergence

// Per-slot iteration state.  Written only by the stop decision (thread 0 of
// k_finalize or of the extra workgroup of a column / forward y pass, after the
// fixed-order reduction of a residual pass), and read at the start of every
// kernel with device-coherent loads (rd_dev.h).
struct State {
    // the four fields every launch branches on come first, in two 8-byte words
    int done;          // inner loop finished (FP64 path: the whole step)
    int iters;         // iterations of the current (inner) PDHG loop
    int outer;         // mixed: outer passes completed
    int outer_done;    // mixed: step finished
    int total_iters;   // mixed: inner iterations summed over outer passes
    int status;        // ST_*
    int inner_best_it; // mixed: inner iteration of the last 10% drop of the inner norm
    int pad;
    double res;        // latest ||F/h_t|| of the current loop (FP64 path: paper norm)
    double res0;       // paper norm at U_0
    double outer_res;  // mixed: latest FP64 paper norm
    double inner_target;
    double mass;       // sum(U - U^k) at the latest FP64 residual evaluation
    double inner_res;
    double inner_best; // mixed: inner norm at inner_best_it
};

// The inner FP32 loop also ends when its norm has not dropped by INNER_DROP for
// INNER_STALL iterations: it has reached the FP32 round-off floor of F~, and
// further iterations cannot help the outer FP64 correction.
constexpr int INNER_STALL = 32;
constexpr double INNER_DROP = 0.9;

struct Slot {
    int N, ncomp, bc, eq;
    int mode, max_iter, max_outer, init;
    int nblk_rows, pad0, pad1, pad2;
    double ht, h, inv_h2, inv_h4;
    double diff[2];
    double b;                    // Allen-Cahn / Cahn-Hilliard reaction coefficient
    double sa, sb, kappa;        // Schnakenberg a, b, kappa
    double tau_u, tau_p, omega, tol, inner_rtol;
    double alpha[2], beta[2];    // G = (I - alpha Lap + beta Lap^2 - gamma Lap^3)^2 per component
    double gamma[2];
    // Iterate buffers, element type T of the PDHG loop (double for FP64, float for
    // the mixed inner loop), each [ncomp][N][N]:
    void *U[2];                  // FP64: U_n ping-pong; mixed: correction e_n ping-pong
    void *P, *Pt;                // dual variable and its extrapolation
    void *S;                     // spectrum, [ncomp][N/2][N] complex, transposed
    double *Uk;                  // U^k (FP64)
    double *U64[2];              // mixed: FP64 U ping-pong across outer passes
    float *r32, *Ub32;           // mixed: FP32 outer residual and FP32 copy of U
    const double *src;           // caller's u_n
    double *partials;            // [nblk_rows][2 * ncomp]
    const double *eig;           // s_k, k < N, for this (N, bc, h)
    const void *tw;              // exp(-2 pi i k / N), k < N, complex T
    const void *twd;             // exp(-i pi k / (2N)), k < N, complex T
    State *st;
};

// ---------------------------------------------------------------- kinds of row-forward pass
enum {
    K_INIT64 = 0,     // FP64 path: U_0 from u_n, U^k copy, W_0 = F(U_0)
    K_ITER64 = 1,     // FP64 path: W_{n+1} = F(U_{n+1})
    K_INNER32 = 2,    // mixed: W = F~(e_{n+1}) in FP32
    K_OUTER_INIT = 3, // mixed: U from u_n, r = F(U) in FP64, inner loop starts
    K_OUTER_UPD = 4,  // mixed: U += e (FP64), r = F(U) in FP64, next inner loop
    K_MIXED = 5       // mixed iteration pass: K_INNER32 while the inner loop runs,
                      // K_OUTER_UPD once it has stopped (read from the State)
};

// ---------------------------------------------------------------- stop decision
// The step's stop rule (Sec. 2.1, stopping criterion; Algorithm 1), its
// iteration limits, and the mixed path's inner-loop rule.
struct StopRule {
    double tol, inner_rtol;
    int max_iter, max_outer;
};

// The State after a residual pass of kind KIND whose norm ||F/h_t|| (summed over
// components) is res and whose sum(U - U^k) is mass.  One pure function, so that
// the same rule runs on the device and in the host-only checks.
//   K_INIT64 / K_ITER64: the FP64 step stops at res <= tol (0 iterations
//     possible), at max_iter, or as non-finite / diverging (res > 1e8 res0).
//   K_INNER32: the FP32 inner loop stops at its target, at max_iter, or after
//     INNER_STALL iterations without a 10 % drop of its norm.
//   K_OUTER_INIT / K_OUTER_UPD: the FP64 outer test of the mixed step, which
//     either ends the step or starts the next inner loop (target
//     max(inner_rtol res, tol / 2)).
//   K_MIXED: K_OUTER_UPD if the inner loop had stopped before the pass, else
//     K_INNER32 (the pass made the outer update iff it had).
// done / outer_done only ever go from 0 to 1 within an inner loop / a step,
// except that an outer decision that continues the step starts a new inner loop
// (done = 0); a launch's workgroups that read the State while the decision is
// being written therefore disagree only where the pass's output is dead.
RD_HD inline bool finite_d(double x) { return x == x && x - x == 0.0; }

template <int KIND> RD_HD inline State decide(const State &in, const StopRule &r, double res, double mass) {
    if constexpr (KIND == K_MIXED) {
        return in.done ? decide<K_OUTER_UPD>(in, r, res, mass) : decide<K_INNER32>(in, r, res, mass);
    }
    State st = in;
    const bool fin = finite_d(res);
    if constexpr (KIND == K_INIT64) {
        st.iters = 0;
        st.total_iters = 0;
        st.outer = 0;
        st.res = res;
        st.res0 = res;
        st.outer_res = res;
        st.mass = mass;
        int done = 1, status = ST_OK;
        if (!fin) status = ST_NONFINITE;
        else if (res <= r.tol) status = ST_OK;
        else if (r.max_iter <= 0) status = ST_NOCONV;
        else done = 0;
        st.status = status;
        st.done = done;
        st.outer_done = done;
    } else if constexpr (KIND == K_ITER64) {
        const int it = in.iters + 1;
        st.iters = it;
        st.total_iters = it;
        st.res = res;
        st.outer_res = res;
        st.mass = mass;
        int done = 1, status = ST_OK;
        if (!fin || res > GROWTH_LIMIT * in.res0) status = ST_NONFINITE;
        else if (res <= r.tol) status = ST_OK;
        else if (it >= r.max_iter) status = ST_NOCONV;
        else done = 0;
        st.status = status;
        st.done = done;
        st.outer_done = done;
    } else if constexpr (KIND == K_INNER32) {
        const int it = in.iters + 1;
        st.iters = it;
        st.total_iters = in.total_iters + 1;
        st.inner_res = res;
        if (!fin) {
            st.status = ST_NONFINITE;
            st.outer_done = 1;
            st.done = 1;
        } else {
            int best_it = in.inner_best_it;
            if (res < INNER_DROP * in.inner_best) {
                st.inner_best = res;
                best_it = it;
                st.inner_best_it = it;
            }
            if (res <= in.inner_target || it >= r.max_iter || it - best_it >= INNER_STALL) st.done = 1;
        }
    } else {
        int outer = 0;
        if constexpr (KIND == K_OUTER_INIT) {
            st.total_iters = 0;
            st.res0 = res;
        } else {
            outer = in.outer + 1;
        }
        st.outer = outer;
        st.outer_res = res;
        st.res = res;
        st.mass = mass;
        int odone = 1, status = ST_OK;
        if (!fin || res > GROWTH_LIMIT * st.res0) status = ST_NONFINITE;
        else if (res <= r.tol) status = ST_OK;
        else if (outer >= r.max_outer || r.max_iter <= 0) status = ST_NOCONV;
        else odone = 0;
        st.status = status;
        st.outer_done = odone;
        st.done = odone;
        st.iters = 0;
        st.inner_target = fmax(r.inner_rtol * res, 0.5 * r.tol);
        st.inner_best = res;
        st.inner_best_it = 0;
    }
    return st;
}

}  // namespace rdk
