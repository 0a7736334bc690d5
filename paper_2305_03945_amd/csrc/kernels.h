// HIP kernels of one G-prox PDHG iteration (Algorithm 1) and of the FP64 outer
// residual passes of the mixed-precision step.
//
// One iteration n -> n+1 is four launches over every active slot:
//   k_cols       column pass of Y = G^-1 W_n: forward column FFT, multiply by
//                1 / (N^2 g), inverse column FFT, in place on the spectrum S
//                (the row pass before it left S = row transforms of W_n).
//   k_rowinv     inverse row transform -> Y_n;  P_{n+1} = P_n + tau_p Y_n,
//                P~ = P_{n+1} + omega (P_{n+1} - P_n)   (eqs. 21-22)
//   k_upd        U_{n+1} = U_n - tau_u grad F(U_n)^T P~ (eq. 23 / 32 / Sec. 3.4.1),
//                reaction derivative at the old U_n
//   k_row_forward W_{n+1} = F(U_{n+1}), per-workgroup partial sums of its squared
//                norm, the forward row transform into S.
// The stop decision for the row pass (Sec. 2.1 stopping criterion) is taken by
// one extra workgroup of the next column pass, which reduces the partial sums
// in a fixed order while the other workgroups transform; after the initial pass
// and at the end of a chunk of iterations, by k_finalize.
// Mixed precision (2-D): the row pass reads from the State which pass the step
// needs.  While the inner FP32 loop runs it is the inner iteration's; once the
// inner loop has stopped, the next row-pass launch makes the FP64 outer update
// instead (U += e, r = F(U), forward transform of r) and the decision after it
// is the outer one, which either ends the step or starts the next inner loop
// on the spectrum of r.  So one fixed launch sequence serves every split of a
// step into inner loops, and the host needs to predict only its total length.
// Every kernel first reads the slot's State and returns at once when it has
// nothing to do, so a host may enqueue more iterations than needed.
#pragma once
#include "fft16.h"

namespace rdk {

// ---------------------------------------------------------------- pointwise reaction prox
// Implicit reaction-only step at one point (predictor for U_0): Allen-Cahn
// u + h_t b (u^3 - u) = c by Newton from u = c (strictly increasing when
// h_t b < 1); Schnakenberg by eliminating v and Newton on u.  Each Newton loop
// stops once a step moves u by at most 2^-50 |u| (from there the quadratic
// convergence has reached round-off; 3-6 steps for |c| <= 1) or after
// PROX_MAX_NEWTON steps, a bound only far-out inputs approach.
constexpr int PROX_MAX_NEWTON = 40;
__device__ __forceinline__ bool newton_converged(double d, double u) { return !(fabs(d) > 0x1p-50 * fabs(u)); }

__device__ __forceinline__ double prox_ac(double c, double ht, double b) {
    const double al = ht * b, be = 1.0 - ht * b;
    double u = c;
#pragma unroll 1
    for (int i = 0; i < PROX_MAX_NEWTON; ++i) {
        const double d = (al * u * u * u + be * u - c) / (3.0 * al * u * u + be);
        u -= d;
        if (newton_converged(d, u)) break;
    }
    return u;
}
// prox_ac at every value of a stencil window (the values load_win reads: row dy
// holds 4 + 2 (HY - |dy|) of them), all advanced by one Newton loop that stops
// when every value has converged.  One loop rather than one per value keeps the
// initial row pass within its register budget (no scratch spills).
template <int HY>
__device__ __forceinline__ void prox_ac_win(double (&v)[2 * HY + 1][4 + 2 * HY], double ht, double b) {
    const double al = ht * b, be = 1.0 - ht * b;
    double c[2 * HY + 1][4 + 2 * HY];
#pragma unroll
    for (int i = 0; i < 2 * HY + 1; ++i) {
        const int hx = HY - (i < HY ? HY - i : i - HY);
#pragma unroll
        for (int j = HY - hx; j < HY + 4 + hx; ++j) c[i][j] = v[i][j];
    }
#pragma unroll 1
    for (int n = 0; n < PROX_MAX_NEWTON; ++n) {
        bool conv = true;
#pragma unroll
        for (int i = 0; i < 2 * HY + 1; ++i) {
            const int hx = HY - (i < HY ? HY - i : i - HY);
#pragma unroll
            for (int j = HY - hx; j < HY + 4 + hx; ++j) {
                const double u = v[i][j];
                const double d = (al * u * u * u + be * u - c[i][j]) / (3.0 * al * u * u + be);
                v[i][j] = u - d;
                conv = conv && newton_converged(d, v[i][j]);
            }
        }
        if (conv) break;
    }
}
__device__ __forceinline__ void prox_schnak(double cu, double cv, double ht, double a, double b, double kap,
                                            double &u, double &v) {
    const double gam = ht * kap, B = cv + gam * b;
    u = cu;
#pragma unroll 1
    for (int i = 0; i < PROX_MAX_NEWTON; ++i) {
        const double dd = 1.0 + gam * u * u;
        const double phi = u - cu - gam * (a - u + u * u * B / dd);
        const double dphi = 1.0 + gam - gam * B * 2.0 * u / (dd * dd);
        const double d = phi / dphi;
        u -= d;
        if (newton_converged(d, u)) break;
    }
    v = B / (1.0 + gam * u * u);
}

// ---------------------------------------------------------------- equation residuals
// Field accessors return the value of component c at (y + dy, x + dx) with the
// boundary mapping already applied by the caller-provided functor.

// F(U) in precision V (Sec. 2.1 eq. 12; Sec. 3.2 eq. 29 with the PDE's sign of the
// biharmonic term; Sec. 3.4.1).  ukc: U^k at the point, per component.
template <int EQ, typename V, class Acc>
__device__ __forceinline__ void eval_F(SlotRef s, Acc u, const V *ukc, V *W, V *Uc) {
    const V ht = (V)s.ht, ih2 = (V)s.inv_h2;
    if constexpr (EQ == EQ_LAP5) {
        const V u0 = u(0, 0, 0);
        const V lap = (u(0, 0, -1) + u(0, 0, 1) + u(0, -1, 0) + u(0, 1, 0) - (V)4 * u0) * ih2;
        const V b = (V)s.b;
        W[0] = u0 - ukc[0] - ht * ((V)s.diff[0] * lap + b * (u0 - u0 * u0 * u0));
        Uc[0] = u0;
    } else if constexpr (EQ == EQ_BIH) {
        const V u0 = u(0, 0, 0);
        const V ul = u(0, 0, -1), ur = u(0, 0, 1), uu = u(0, -1, 0), ud = u(0, 1, 0);
        const V axis1 = ul + ur + uu + ud;
        const V diag = u(0, -1, -1) + u(0, -1, 1) + u(0, 1, -1) + u(0, 1, 1);
        const V axis2 = u(0, 0, -2) + u(0, 0, 2) + u(0, -2, 0) + u(0, 2, 0);
        const V lap13 = ((V)20 * u0 - (V)8 * axis1 + (V)2 * diag + axis2) * (V)s.inv_h4;
        const V b = (V)s.b;
        auto g = [b](V v) { return b * (v * v * v - v); };
        const V lapg = (g(ul) + g(ur) + g(uu) + g(ud) - (V)4 * g(u0)) * ih2;
        W[0] = u0 - ukc[0] + (V)s.diff[0] * ht * lap13 - ht * lapg;
        Uc[0] = u0;
    } else if constexpr (EQ == EQ_FCH) {
        // Sec. 3.3: mu = eps^2 Lap U - W1(U), nu = eps^2 Lap mu - W2(U) mu + eps^2 mu,
        // F = U - U^k - h_t Lap nu; W1 = u^3 - u, W2 = 3u^2 - 1.  Evaluated from U on
        // the 25-point neighbourhood (the compiler shares the repeated sub-terms).
        const V e2 = (V)s.diff[0];
        auto lapu = [&](int dy, int dx) {
            return (u(0, dy, dx - 1) + u(0, dy, dx + 1) + u(0, dy - 1, dx) + u(0, dy + 1, dx) - (V)4 * u(0, dy, dx)) * ih2;
        };
        auto mu = [&](int dy, int dx) {
            const V v = u(0, dy, dx);
            return e2 * lapu(dy, dx) - (v * v * v - v);
        };
        auto nu = [&](int dy, int dx) {
            const V v = u(0, dy, dx), m = mu(dy, dx);
            const V lapm = (mu(dy, dx - 1) + mu(dy, dx + 1) + mu(dy - 1, dx) + mu(dy + 1, dx) - (V)4 * m) * ih2;
            return e2 * lapm - ((V)3 * v * v - (V)1) * m + e2 * m;
        };
        const V lapnu = (nu(0, -1) + nu(0, 1) + nu(-1, 0) + nu(1, 0) - (V)4 * nu(0, 0)) * ih2;
        const V u0 = u(0, 0, 0);
        W[0] = u0 - ukc[0] - ht * lapnu;
        Uc[0] = u0;
    } else {
        const V u0 = u(0, 0, 0), v0 = u(1, 0, 0);
        const V lu = (u(0, 0, -1) + u(0, 0, 1) + u(0, -1, 0) + u(0, 1, 0) - (V)4 * u0) * ih2;
        const V lv = (u(1, 0, -1) + u(1, 0, 1) + u(1, -1, 0) + u(1, 1, 0) - (V)4 * v0) * ih2;
        const V kap = (V)s.kappa, u2v = u0 * u0 * v0;
        W[0] = u0 - ukc[0] - ht * ((V)s.diff[0] * lu + kap * ((V)s.sa - u0 + u2v));
        W[1] = v0 - ukc[1] - ht * ((V)s.diff[1] * lv + kap * ((V)s.sb - u2v));
        Uc[0] = u0;
        Uc[1] = v0;
    }
}

// F~(e) = F(U + e) for the mixed inner loop, written as r + (linear part) e minus
// h_t times the exact reaction difference, expanded so that no difference of two
// nearly equal FP32 numbers is formed:
//   Allen-Cahn:   f(U+e) - f(U) = b (e - 3U^2 e - 3U e^2 - e^3)
//   Cahn-Hilliard: g(U+e) - g(U) = b (3U^2 e + 3U e^2 + e^3 - e)  (under Lap)
//   Schnakenberg: (U+e_u)^2 (V+e_v) - U^2 V = 2UV e_u + U^2 e_v + V e_u^2 + 2U e_u e_v + e_u^2 e_v
//   FCH (Sec. 3.3): with mu(U) = eps^2 Lap U - W1(U), nu = eps^2 Lap mu - W2(U) mu + eps^2 mu,
//     d_mu = eps^2 Lap e - (W1(U+e) - W1(U)),  W1(U+e) - W1(U) = 3U^2 e + 3U e^2 + e^3 - e,
//     d_nu = eps^2 Lap d_mu + eps^2 d_mu - W2(U+e) d_mu - (W2(U+e) - W2(U)) mu(U),
//     W2(U+e) - W2(U) = 6U e + 3e^2,  and F~ = r + e - h_t Lap d_nu
//   (e on the 25-point reach, U on the 13-point one).
// e: accessor of the correction, ub: accessor of the FP32 copy of U.
template <int EQ, class AccE, class AccU>
__device__ __forceinline__ void eval_Ftilde(SlotRef s, AccE e, AccU ub, const float *rc, float *W) {
    const float ht = (float)s.ht, ih2 = (float)s.inv_h2;
    if constexpr (EQ == EQ_LAP5) {
        const float e0 = e(0, 0, 0), U = ub(0, 0, 0);
        const float lap = (e(0, 0, -1) + e(0, 0, 1) + e(0, -1, 0) + e(0, 1, 0) - 4.0f * e0) * ih2;
        const float df = (float)s.b * (e0 - 3.0f * U * U * e0 - 3.0f * U * e0 * e0 - e0 * e0 * e0);
        W[0] = rc[0] + e0 - ht * ((float)s.diff[0] * lap + df);
    } else if constexpr (EQ == EQ_BIH) {
        const float e0 = e(0, 0, 0);
        const float el = e(0, 0, -1), er = e(0, 0, 1), eu = e(0, -1, 0), ed = e(0, 1, 0);
        const float axis1 = el + er + eu + ed;
        const float diag = e(0, -1, -1) + e(0, -1, 1) + e(0, 1, -1) + e(0, 1, 1);
        const float axis2 = e(0, 0, -2) + e(0, 0, 2) + e(0, -2, 0) + e(0, 2, 0);
        const float lap13 = (20.0f * e0 - 8.0f * axis1 + 2.0f * diag + axis2) * (float)s.inv_h4;
        const float b = (float)s.b;
        auto dg = [b](float U, float d) { return b * (3.0f * U * U * d + 3.0f * U * d * d + d * d * d - d); };
        const float lapdg = (dg(ub(0, 0, -1), el) + dg(ub(0, 0, 1), er) + dg(ub(0, -1, 0), eu) +
                             dg(ub(0, 1, 0), ed) - 4.0f * dg(ub(0, 0, 0), e0)) * ih2;
        W[0] = rc[0] + e0 + (float)s.diff[0] * ht * lap13 - ht * lapdg;
    } else if constexpr (EQ == EQ_FCH) {
        const float e2 = (float)s.diff[0];
        auto ev = [&](int dy, int dx) { return e(0, dy, dx); };
        auto uv = [&](int dy, int dx) { return ub(0, dy, dx); };
        auto lap = [&](auto f, int dy, int dx) {
            return (f(dy, dx - 1) + f(dy, dx + 1) + f(dy - 1, dx) + f(dy + 1, dx) - 4.0f * f(dy, dx)) * ih2;
        };
        auto dmu = [&](int dy, int dx) {
            const float E = ev(dy, dx), U = uv(dy, dx);
            return e2 * lap(ev, dy, dx) - (3.0f * U * U * E + 3.0f * U * E * E + E * E * E - E);
        };
        auto dnu = [&](int dy, int dx) {
            const float E = ev(dy, dx), U = uv(dy, dx), d = dmu(dy, dx), V = U + E;
            const float muU = e2 * lap(uv, dy, dx) - (U * U * U - U);
            return e2 * lap(dmu, dy, dx) + e2 * d - (3.0f * V * V - 1.0f) * d - (6.0f * U * E + 3.0f * E * E) * muU;
        };
        W[0] = rc[0] + ev(0, 0) - ht * lap(dnu, 0, 0);
    } else {
        const float eu0 = e(0, 0, 0), ev0 = e(1, 0, 0);
        const float U = ub(0, 0, 0), Vv = ub(1, 0, 0);
        const float lu = (e(0, 0, -1) + e(0, 0, 1) + e(0, -1, 0) + e(0, 1, 0) - 4.0f * eu0) * ih2;
        const float lv = (e(1, 0, -1) + e(1, 0, 1) + e(1, -1, 0) + e(1, 1, 0) - 4.0f * ev0) * ih2;
        const float d = 2.0f * U * Vv * eu0 + U * U * ev0 + Vv * eu0 * eu0 + 2.0f * U * eu0 * ev0 + eu0 * eu0 * ev0;
        const float kap = (float)s.kappa;
        W[0] = rc[0] + eu0 - ht * ((float)s.diff[0] * lu + kap * (-eu0 + d));
        W[1] = rc[1] + ev0 - ht * ((float)s.diff[1] * lv - kap * d);
    }
}

// grad F(U)^T P~ at one point (eq. 23; eq. 32 with the PDE's sign; Sec. 3.4.1).
// p: accessor of P~; Uc: U at the point per component.
template <int EQ, typename V, class Acc>
__device__ __forceinline__ void eval_adjoint(SlotRef s, Acc p, const V *Uc, V *out) {
    const V ht = (V)s.ht, ih2 = (V)s.inv_h2;
    if constexpr (EQ == EQ_LAP5) {
        const V p0 = p(0, 0, 0);
        const V lap = (p(0, 0, -1) + p(0, 0, 1) + p(0, -1, 0) + p(0, 1, 0) - (V)4 * p0) * ih2;
        const V U = Uc[0];
        out[0] = p0 - (V)s.diff[0] * ht * lap - ht * ((V)s.b * ((V)1 - (V)3 * U * U)) * p0;
    } else if constexpr (EQ == EQ_BIH) {
        const V p0 = p(0, 0, 0);
        const V axis1 = p(0, 0, -1) + p(0, 0, 1) + p(0, -1, 0) + p(0, 1, 0);
        const V diag = p(0, -1, -1) + p(0, -1, 1) + p(0, 1, -1) + p(0, 1, 1);
        const V axis2 = p(0, 0, -2) + p(0, 0, 2) + p(0, -2, 0) + p(0, 2, 0);
        const V lap13 = ((V)20 * p0 - (V)8 * axis1 + (V)2 * diag + axis2) * (V)s.inv_h4;
        const V lap5 = (axis1 - (V)4 * p0) * ih2;
        const V U = Uc[0];
        out[0] = p0 + (V)s.diff[0] * ht * lap13 - ht * ((V)s.b * ((V)3 * U * U - (V)1)) * lap5;
    } else {
        const V p0 = p(0, 0, 0), q0 = p(1, 0, 0);
        const V lp = (p(0, 0, -1) + p(0, 0, 1) + p(0, -1, 0) + p(0, 1, 0) - (V)4 * p0) * ih2;
        const V lq = (p(1, 0, -1) + p(1, 0, 1) + p(1, -1, 0) + p(1, 1, 0) - (V)4 * q0) * ih2;
        const V U = Uc[0], Vv = Uc[1], kap = (V)s.kappa;
        out[0] = p0 - ht * ((V)s.diff[0] * lp + kap * (-p0 + (V)2 * U * Vv * (p0 - q0)));
        out[1] = q0 - ht * ((V)s.diff[1] * lq + kap * U * U * (p0 - q0));
    }
}

// grad F(U)^T P~ of the FCH step (Sec. 3.3): with q = Lap P~, D = W2(U),
// B = eps^2 Lap U - W1(U):
//   out = P~ - h_t (eps^2 Lap - D)(eps^2 Lap - D + eps^2) q + h_t W3(U) B q.
// p: accessor of P~ (25-point reach), u: accessor of U (5-point reach).
template <typename V, class AccP, class AccU>
__device__ __forceinline__ V eval_adjoint_fch(SlotRef s, AccP p, AccU u) {
    const V ht = (V)s.ht, ih2 = (V)s.inv_h2, e2 = (V)s.diff[0];
    auto q = [&](int dy, int dx) {
        return (p(0, dy, dx - 1) + p(0, dy, dx + 1) + p(0, dy - 1, dx) + p(0, dy + 1, dx) - (V)4 * p(0, dy, dx)) * ih2;
    };
    auto a = [&](int dy, int dx) {
        const V v = u(0, dy, dx), qq = q(dy, dx);
        const V lapq = (q(dy, dx - 1) + q(dy, dx + 1) + q(dy - 1, dx) + q(dy + 1, dx) - (V)4 * qq) * ih2;
        return e2 * lapq - ((V)3 * v * v - (V)1) * qq + e2 * qq;
    };
    const V u0 = u(0, 0, 0), a0 = a(0, 0);
    const V lapa = (a(0, -1) + a(0, 1) + a(-1, 0) + a(1, 0) - (V)4 * a0) * ih2;
    const V lapu = (u(0, 0, -1) + u(0, 0, 1) + u(0, -1, 0) + u(0, 1, 0) - (V)4 * u0) * ih2;
    const V B = e2 * lapu - (u0 * u0 * u0 - u0);
    return p(0, 0, 0) - ht * (e2 * lapa - ((V)3 * u0 * u0 - (V)1) * a0) + ht * ((V)6 * u0) * B * q(0, 0);
}

// ---------------------------------------------------------------- stencil windows
// Four consecutive points (y, x0 .. x0+3) of one row, x0 a multiple of 4, with
// the stencil neighbourhood they need: row y + dy holds x0 - hx .. x0 + 3 + hx,
// hx = HY - |dy| (HY = 1: the 5-point stencil; HY = 2: the 13-point one; HY = 0:
// the four points only).  The four middle values are one aligned vector load;
// the edge values are scalar loads through the boundary map.
template <typename T> using vec4_t = T __attribute__((ext_vector_type(4)));

template <typename T, int HY> struct Win {
    T v[2 * HY + 1][4 + 2 * HY];
    __device__ __forceinline__ T at(int k, int dy, int dx) const { return v[dy + HY][HY + dx + k]; }
};

template <typename T, int BC, int LOGN, int HY>
__device__ __forceinline__ void load_win(Win<T, HY> &w, gptr_t<const T> f, int y, int x0) {
    constexpr int N = 1 << LOGN;
#pragma unroll
    for (int dy = -HY; dy <= HY; ++dy) {
        const int hx = HY - (dy < 0 ? -dy : dy);
        const gptr_t<const T> row = f + (size_t)wrap<BC>(y + dy, N) * N;
        const vec4_t<T> m = *(const gptr_t<const vec4_t<T>>)(row + x0);
#pragma unroll
        for (int k = 0; k < 4; ++k) w.v[dy + HY][HY + k] = m[k];
#pragma unroll
        for (int h = 1; h <= hx; ++h) {
            w.v[dy + HY][HY - h] = row[wrap<BC>(x0 - h, N)];
            w.v[dy + HY][HY + 3 + h] = row[wrap<BC>(x0 + 3 + h, N)];
        }
    }
}

// Window of two adjacent rows y, y + 1 (four points each) for a stencil of reach
// HY: rows y - HY .. y + 1 + HY, each with the x-halo that an output row at its
// distance needs.  Shared rows are loaded once.
template <typename T, int HY> struct Win2 {
    T v[2 * HY + 2][4 + 2 * HY];
    // row j (0: y, 1: y + 1) of the output pair
    __device__ __forceinline__ T at(int j, int k, int dy, int dx) const { return v[j + dy + HY][HY + dx + k]; }
};

template <typename T, int BC, int LOGN, int HY>
__device__ __forceinline__ void load_win2(Win2<T, HY> &w, gptr_t<const T> f, int y, int x0) {
    constexpr int N = 1 << LOGN;
#pragma unroll
    for (int d = -HY; d <= HY + 1; ++d) {
        const int dist = d < 0 ? -d : (d > 1 ? d - 1 : 0);   // to the nearer output row
        const int hx = HY - dist;
        const gptr_t<const T> row = f + (size_t)wrap<BC>(y + d, N) * N;
        const vec4_t<T> m = *(const gptr_t<const vec4_t<T>>)(row + x0);
#pragma unroll
        for (int k = 0; k < 4; ++k) w.v[d + HY][HY + k] = m[k];
#pragma unroll
        for (int h = 1; h <= hx; ++h) {
            w.v[d + HY][HY - h] = row[wrap<BC>(x0 - h, N)];
            w.v[d + HY][HY + 3 + h] = row[wrap<BC>(x0 + 3 + h, N)];
        }
    }
}

template <typename T> __device__ __forceinline__ vec4_t<T> load4(gptr_t<const T> p) {
    return *(const gptr_t<const vec4_t<T>>)p;
}
template <typename T> __device__ __forceinline__ void store4(gptr_t<T> p, const vec4_t<T> &v) {
    *(gptr_t<vec4_t<T>>)p = v;
}

template <int EQ> constexpr int stencil_hy() { return EQ == EQ_FCH ? 3 : EQ == EQ_BIH ? 2 : 1; }
// Reach of the FP32 copy of U in the mixed inner residual: Cahn-Hilliard needs it at
// the 5-point neighbours (reaction under Lap), FCH on the 13-point neighbourhood
// (mu(U) under Lap, and the reaction difference under Lap^2); the others at the point.
template <int EQ> constexpr int ftilde_hu() { return EQ == EQ_FCH ? 2 : EQ == EQ_BIH ? 1 : 0; }

// ---------------------------------------------------------------- deterministic block sums
// Workgroup sum of K values per thread, in a fixed order (wave butterflies, then
// the waves in order); the totals are valid in thread 0 only.
template <int K> __device__ __forceinline__ void block_sum(double *v, double *scratch /* K * NT/64 */) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        v[k] = x;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) scratch[k * (NT / 64) + wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double x = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) x += scratch[k * (NT / 64) + w];
            v[k] = x;
        }
    }
}

// Slot stop decision after a residual reduction (thread 0 of the deciding
// workgroup): the decision rule of rd_types.h on the State read coherently.
template <int KIND, int C>
__device__ __forceinline__ void finalize(SlotRef s, const double *sumsq, const double *mass) {
    double res = 0.0, m = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        res += sqrt(sumsq[c]);
        m += mass[c];
    }
    res /= s.ht;
    State *st = s.st;
    const StopRule rule{s.tol, s.inner_rtol, s.max_iter, s.max_outer};
    store_state(st, decide<KIND>(load_state(st), rule, res, m));
}

// Write this workgroup's partial sums (squared residual norm and sum(U - U^k)
// per component) to the slot's partials array.  The stop decision is taken by
// k_finalize, launched right after, which reads them after the kernel boundary.
template <int C>
__device__ __forceinline__ void write_partials(SlotRef s, int tile, double *acc /* 2C */, double *scratch) {
    block_sum<2 * C>(acc, scratch);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 2 * C; ++k) s.partials[tile * (2 * C) + k] = acc[k];
    }
}

// Whether a launch of this kind has nothing to do for the slot (same answer in
// every wave: the State does not change during the launch).
template <int KIND> __device__ __forceinline__ bool skip_launch(StateRef sst) {
    if constexpr (KIND == K_INIT64 || KIND == K_OUTER_INIT) return false;
    else if constexpr (KIND == K_OUTER_UPD) return sst.outer_done || !sst.done;
    else if constexpr (KIND == K_MIXED) return sst.outer_done != 0;
    else return sst.done != 0;
}

// ---------------------------------------------------------------- stop decision
// Sum of the row pass's per-workgroup partials in one fixed order, whatever the
// size of the workgroup that computes it: 64 lane sums L_l = sum_j p[l + 64 j]
// (j increasing), then sum_l L_l (l increasing) by thread 0.  The decision is
// taken either by k_finalize or by the extra workgroup of a column pass; both
// give bitwise the same sums.  lanes: LDS scratch of 64 * 2C doubles.
template <int KIND, int C, int NTHR>
__device__ __forceinline__ void reduce_and_finalize(SlotRef s, double *lanes) {
    constexpr int K = 2 * C;
    const int nb = s.nblk_rows;
    const auto part = gp((const double *)s.partials);
    for (int l = threadIdx.x; l < 64; l += NTHR) {
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = 0.0;
        for (int j = l; j < nb; j += 64) {
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] += part[j * K + k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) lanes[k * 64 + l] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double x = 0.0;
            for (int l = 0; l < 64; ++l) x += lanes[k * 64 + l];
            v[k] = x;
        }
        finalize<KIND, C>(s, v, v + C);
    }
}

// One workgroup per slot: the stop decision of the row pass of kind KIND.  Skips
// exactly when the row-pass launch of the same kind skipped.
template <int KIND, int C>
__global__ __launch_bounds__(NT) void k_finalize(Slot *const *slots) {
    __shared__ double lanes[64 * 2 * C];
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if (skip_launch<KIND>(sst)) return;
    reduce_and_finalize<KIND, C, NT>(s, lanes);
}

// The residual-type quantity a row-forward pass transforms, on four consecutive
// points (y, x0..x0+3) with vector loads: wv[k][c] receives, for every
// component, W = F(U) (FP64 kinds) or the FP32 inner residual F~(e) at point k;
// acc[c] accumulates the squared norm and acc[C + c] sum(U - U^k).  The kinds'
// side effects: the initial kinds store U_0 and U^k, the mixed outer kinds store
// the FP64 U, its FP32 copy and the FP32 residual r.
template <typename T, int LOGN, int BC, int EQ, int KIND>
__device__ __forceinline__ void produce_W4(SlotRef s, StateRef sst, int y, int x0, T (*wv)[EQ == EQ_SCHNAK ? 2 : 1],
                                           double *acc) {
    constexpr int N = 1 << LOGN;
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr size_t NN = (size_t)N * N;
    constexpr int HY = stencil_hy<EQ>();
    const int it = sst.iters;
    const size_t g0 = (size_t)y * N + x0;
    if constexpr (KIND != K_INNER32) {
        // FP64 kinds: the iterate U (window wu) and U^k at the four points
        Win<double, HY> wu[C];
        vec4_t<double> uk[C];
        if constexpr (KIND == K_ITER64) {
            const auto Un = gp((const double *)s.U[(it + 1) & 1]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                load_win<double, BC, LOGN, HY>(wu[c], Un + c * NN, y, x0);
                uk[c] = load4<double>(gp((const double *)s.Uk) + c * NN + g0);
            }
        } else if constexpr (KIND == K_INIT64 || KIND == K_OUTER_INIT) {
            // U_0 = U^k, or the pointwise reaction prox of U^k (predictor)
            const auto src = gp(s.src);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                load_win<double, BC, LOGN, HY>(wu[c], src + c * NN, y, x0);
#pragma unroll
                for (int k = 0; k < 4; ++k) uk[c][k] = wu[c].at(k, 0, 0);
            }
            if (s.init != 0) {
                if constexpr (EQ == EQ_LAP5) {
                    prox_ac_win<HY>(wu[0].v, s.ht, s.b);
                } else if constexpr (EQ == EQ_SCHNAK) {
#pragma unroll
                    for (int i = 0; i < 2 * HY + 1; ++i) {
                        const int hx = HY - (i < HY ? HY - i : i - HY);
#pragma unroll
                        for (int j = HY - hx; j < HY + 4 + hx; ++j) {
                            double u, v;
                            prox_schnak(wu[0].v[i][j], wu[1].v[i][j], s.ht, s.sa, s.sb, s.kappa, u, v);
                            wu[0].v[i][j] = u;
                            wu[1].v[i][j] = v;
                        }
                    }
                }
            }
        } else {
            // mixed outer update: U = U_prev + e (e absent before the first inner iteration)
            const auto Ucur = gp((const double *)s.U64[sst.outer & 1]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                load_win<double, BC, LOGN, HY>(wu[c], Ucur + c * NN, y, x0);
                uk[c] = load4<double>(gp((const double *)s.Uk) + c * NN + g0);
            }
            if (sst.iters > 0) {
                const auto E = gp((const float *)s.U[sst.iters & 1]);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    Win<float, HY> we;
                    load_win<float, BC, LOGN, HY>(we, E + c * NN, y, x0);
#pragma unroll
                    for (int i = 0; i < 2 * HY + 1; ++i) {
                        const int hx = HY - (i < HY ? HY - i : i - HY);
#pragma unroll
                        for (int j = HY - hx; j < HY + 4 + hx; ++j) wu[c].v[i][j] += (double)we.v[i][j];
                    }
                }
            }
        }
        vec4_t<double> Uc4[C], W4[C];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double W[C], Uc[C], ukc[C];
#pragma unroll
            for (int c = 0; c < C; ++c) ukc[c] = uk[c][k];
            eval_F<EQ, double>(s, [&](int c, int dy, int dx) { return wu[c].at(k, dy, dx); }, ukc, W, Uc);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                acc[c] += W[c] * W[c];
                acc[C + c] += Uc[c] - ukc[c];
                Uc4[c][k] = Uc[c];
                W4[c][k] = W[c];
                // the mixed inner loop starts from the FP32 residual
                wv[k][c] = (KIND == K_OUTER_INIT || KIND == K_OUTER_UPD) ? (T)(float)W[c] : (T)W[c];
            }
        }
        if constexpr (KIND == K_INIT64 || KIND == K_OUTER_INIT || KIND == K_OUTER_UPD) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if constexpr (KIND == K_INIT64) {
                    store4<double>(gp((double *)s.U[0]) + c * NN + g0, Uc4[c]);
                } else if constexpr (KIND == K_OUTER_INIT) {
                    store4<double>(gp(s.U64[0]) + c * NN + g0, Uc4[c]);
                } else {
                    store4<double>(gp(s.U64[(sst.outer + 1) & 1]) + c * NN + g0, Uc4[c]);
                }
                if constexpr (KIND != K_OUTER_UPD) store4<double>(gp(s.Uk) + c * NN + g0, uk[c]);
                if constexpr (KIND != K_INIT64) {
                    vec4_t<float> r4, ub4;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        r4[k] = (float)W4[c][k];
                        ub4[k] = (float)Uc4[c][k];
                    }
                    store4<float>(gp(s.r32) + c * NN + g0, r4);
                    store4<float>(gp(s.Ub32) + c * NN + g0, ub4);
                }
            }
        }
    } else {
        static_assert(KIND == K_INNER32, "vectorised producer: iteration kinds only");
        constexpr int HU = ftilde_hu<EQ>();
        const auto E = gp((const float *)s.U[(it + 1) & 1]);
        const auto Ub = gp((const float *)s.Ub32);
        Win<float, HY> we[C];
        Win<float, HU> wub[C];
        vec4_t<float> r4[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            load_win<float, BC, LOGN, HY>(we[c], E + c * NN, y, x0);
            load_win<float, BC, LOGN, HU>(wub[c], Ub + c * NN, y, x0);
            r4[c] = load4<float>(gp((const float *)s.r32) + c * NN + g0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float rc[C], W[C];
#pragma unroll
            for (int c = 0; c < C; ++c) rc[c] = r4[c][k];
            eval_Ftilde<EQ>(s, [&](int c, int dy, int dx) { return we[c].at(k, dy, dx); },
                            [&](int c, int dy, int dx) { return wub[c].at(k, dy, dx); }, rc, W);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                acc[c] += (double)W[c] * (double)W[c];
                wv[k][c] = (T)W[c];
            }
        }
    }
}

// produce_W4 for the iteration kinds on two adjacent rows y, y + 1 at once: the
// rows the two stencils share are loaded once.  wv[j][k][c] receives row j's value
// at point k; acc as in produce_W4 (both rows).
template <typename T, int LOGN, int BC, int EQ, int KIND>
__device__ __forceinline__ void produce_W4x2(SlotRef s, StateRef sst, int y, int x0,
                                             T (*wv)[4][EQ == EQ_SCHNAK ? 2 : 1], double *acc) {
    static_assert(KIND == K_ITER64 || KIND == K_INNER32 || KIND == K_OUTER_UPD,
                  "two-row producer: iteration and outer-update kinds");
    constexpr int N = 1 << LOGN;
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr size_t NN = (size_t)N * N;
    constexpr int HY = stencil_hy<EQ>();
    const int it = sst.iters;
    const size_t g0 = (size_t)y * N + x0;
    if constexpr (KIND == K_OUTER_UPD) {
        // U = U_prev + e in FP64 on the two-row window, r = F(U); stores U, its FP32
        // copy and the FP32 r of both rows
        const auto Ucur = gp((const double *)s.U64[sst.outer & 1]);
        Win2<double, HY> wu[C];
        vec4_t<double> uk[2][C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            load_win2<double, BC, LOGN, HY>(wu[c], Ucur + c * NN, y, x0);
#pragma unroll
            for (int j = 0; j < 2; ++j) uk[j][c] = load4<double>(gp((const double *)s.Uk) + c * NN + g0 + j * N);
        }
        if (sst.iters > 0) {
            const auto E = gp((const float *)s.U[sst.iters & 1]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                Win2<float, HY> we;
                load_win2<float, BC, LOGN, HY>(we, E + c * NN, y, x0);
#pragma unroll
                for (int d = 0; d < 2 * HY + 2; ++d) {
                    const int dd = d - HY;   // offset from row y; the loaded x-halo is load_win2's
                    const int hx = HY - (dd < 0 ? -dd : (dd > 1 ? dd - 1 : 0));
#pragma unroll
                    for (int i = HY - hx; i < HY + 4 + hx; ++i) wu[c].v[d][i] += (double)we.v[d][i];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            vec4_t<double> Uc4[C];
            vec4_t<float> r4[C], ub4[C];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double W[C], Uc[C], ukc[C];
#pragma unroll
                for (int c = 0; c < C; ++c) ukc[c] = uk[j][c][k];
                eval_F<EQ, double>(s, [&](int c, int dy, int dx) { return wu[c].at(j, k, dy, dx); }, ukc, W, Uc);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    acc[c] += W[c] * W[c];
                    acc[C + c] += Uc[c] - ukc[c];
                    Uc4[c][k] = Uc[c];
                    r4[c][k] = (float)W[c];
                    ub4[c][k] = (float)Uc[c];
                    wv[j][k][c] = (T)(float)W[c];
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const size_t g = c * NN + g0 + j * N;
                store4<double>(gp(s.U64[(sst.outer + 1) & 1]) + g, Uc4[c]);
                store4<float>(gp(s.r32) + g, r4[c]);
                store4<float>(gp(s.Ub32) + g, ub4[c]);
            }
        }
    } else if constexpr (KIND == K_ITER64) {
        const auto Un = gp((const double *)s.U[(it + 1) & 1]);
        Win2<double, HY> wu[C];
        vec4_t<double> uk[2][C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            load_win2<double, BC, LOGN, HY>(wu[c], Un + c * NN, y, x0);
#pragma unroll
            for (int j = 0; j < 2; ++j) uk[j][c] = load4<double>(gp((const double *)s.Uk) + c * NN + g0 + j * N);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double W[C], Uc[C], ukc[C];
#pragma unroll
                for (int c = 0; c < C; ++c) ukc[c] = uk[j][c][k];
                eval_F<EQ, double>(s, [&](int c, int dy, int dx) { return wu[c].at(j, k, dy, dx); }, ukc, W, Uc);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    acc[c] += W[c] * W[c];
                    acc[C + c] += Uc[c] - ukc[c];
                    wv[j][k][c] = (T)W[c];
                }
            }
    } else {
        constexpr int HU = ftilde_hu<EQ>();
        const auto E = gp((const float *)s.U[(it + 1) & 1]);
        const auto Ub = gp((const float *)s.Ub32);
        Win2<float, HY> we[C];
        Win2<float, HU> wub[C];
        vec4_t<float> r4[2][C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            load_win2<float, BC, LOGN, HY>(we[c], E + c * NN, y, x0);
            load_win2<float, BC, LOGN, HU>(wub[c], Ub + c * NN, y, x0);
#pragma unroll
            for (int j = 0; j < 2; ++j) r4[j][c] = load4<float>(gp((const float *)s.r32) + c * NN + g0 + j * N);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float rc[C], W[C];
#pragma unroll
                for (int c = 0; c < C; ++c) rc[c] = r4[j][c][k];
                eval_Ftilde<EQ>(s, [&](int c, int dy, int dx) { return we[c].at(j, k, dy, dx); },
                                [&](int c, int dy, int dx) { return wub[c].at(j, k, dy, dx); }, rc, W);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    acc[c] += (double)W[c] * (double)W[c];
                    wv[j][k][c] = (T)W[c];
                }
            }
    }
}

// ---------------------------------------------------------------- spectrum layout
// Per component, N^2/2 complex entries: (kx, y) for kx < N/2 the packed row
// spectrum slot (periodic) or cosine pair (Neumann) of row y.  Stored in tiles
// of the row pass's R rows, S[c][y / R][kx][y % R]: a row-pass workgroup writes
// one contiguous block, and a column-pass workgroup that takes CB adjacent
// columns reads CB * R contiguous entries per tile.
template <int R>
__device__ __forceinline__ size_t spec_off(int c, int y, int kx, int N) {
    const size_t H = (size_t)N / 2;
    return (size_t)c * H * N + ((size_t)(y / R) * H + kx) * R + (y % R);
}

// Spectrum entries are moved SV at a time, 16 bytes per access: two FP32
// complex values (rows r, r + 1 of a tile, adjacent in S) or one FP64 value.
template <typename T> constexpr int spec_vec() { return sizeof(T) == 4 ? 2 : 1; }
template <typename T> __device__ __forceinline__ void spec_load(const cplx<T> *p, cplx<T> *out) {
    if constexpr (sizeof(T) == 4) {
        const vec4_t<float> v = load4<float>(gp((const float *)p));
        out[0] = {v[0], v[1]};
        out[1] = {v[2], v[3]};
    } else {
        typedef double v2d __attribute__((ext_vector_type(2)));
        const v2d v = *(const gptr_t<const v2d>)gp((const double *)p);
        out[0] = {v[0], v[1]};
    }
}
template <typename T> __device__ __forceinline__ void spec_store(cplx<T> *p, const cplx<T> *in) {
    if constexpr (sizeof(T) == 4) {
        vec4_t<float> v;
        v[0] = in[0].re;
        v[1] = in[0].im;
        v[2] = in[1].re;
        v[3] = in[1].im;
        store4<float>(gp((float *)p), v);
    } else {
        typedef double v2d __attribute__((ext_vector_type(2)));
        v2d v;
        v[0] = in[0].re;
        v[1] = in[0].im;
        *(gptr_t<v2d>)gp((double *)p) = v;
    }
}

// Periodic rows: the pair spectra of a block's rows go from LDS (after the
// forward transform) straight to the tiles of S, and back.  Item (reg, l), reg
// fastest, owns slot l of the two rows packed in region reg: the rows are
// adjacent in a tile, so the two values are one 16-byte access (FP32) or two
// adjacent ones (FP64), and consecutive items walk the tile contiguously.
// Region reg holds component reg / (R/2), rows 2 (reg % (R/2)) and the next.
template <typename T, int LOGN, int C, int R>
__device__ __forceinline__ cplx<T> *slot_pair(cplx<T> *S, int reg, int y0, int l) {
    return &S[spec_off<R>(reg / (R / 2), y0 + 2 * (reg % (R / 2)), l, 1 << LOGN)];
}

template <typename T, int LOGN, int C, int R, int NTH>
__device__ __forceinline__ void rows_post_store(const cplx<T> *buf, cplx<T> *S, int y0) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int NREG = C * R / 2;
    constexpr int TOT = NREG * H;
#pragma unroll
    for (int i = 0; i < (TOT + NTH - 1) / NTH; ++i) {
        const int it = threadIdx.x + i * NTH;
        if (TOT % NTH != 0 && it >= TOT) break;
        const int reg = it % NREG, l = it / NREG;
        cplx<T> v[2];
        if (l == 0) {
            const cplx<T> z0 = buf[rix<LOGN>(reg, 0)], zh = buf[rix<LOGN>(reg, H)];
            v[0] = {z0.re, zh.re};
            v[1] = {z0.im, zh.im};
        } else {
            const cplx<T> zl = buf[rix<LOGN>(reg, l)], zn = buf[rix<LOGN>(reg, N - l)];
            v[0] = {(zl.re + zn.re) * (T)0.5, (zl.im - zn.im) * (T)0.5};
            v[1] = {(zl.im + zn.im) * (T)0.5, (zn.re - zl.re) * (T)0.5};
        }
        cplx<T> *p = slot_pair<T, LOGN, C, R>(S, reg, y0, l);
        if constexpr (spec_vec<T>() == 2) {
            spec_store<T>(p, v);
        } else {
            spec_store<T>(p, v);
            spec_store<T>(p + 1, v + 1);
        }
    }
}

template <typename T, int LOGN, int C, int R, int NTH>
__device__ __forceinline__ void rows_load_pre(cplx<T> *buf, const cplx<T> *S, int y0) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int NREG = C * R / 2;
    constexpr int TOT = NREG * H;
#pragma unroll
    for (int i = 0; i < (TOT + NTH - 1) / NTH; ++i) {
        const int it = threadIdx.x + i * NTH;
        if (TOT % NTH != 0 && it >= TOT) break;
        const int reg = it % NREG, l = it / NREG;
        const cplx<T> *p = slot_pair<T, LOGN, C, R>(const_cast<cplx<T> *>(S), reg, y0, l);
        cplx<T> v[2];
        if constexpr (spec_vec<T>() == 2) {
            spec_load<T>(p, v);
        } else {
            spec_load<T>(p, v);
            spec_load<T>(p + 1, v + 1);
        }
        const cplx<T> a = v[0], b = v[1];
        if (l == 0) {
            buf[rix<LOGN>(reg, 0)] = {a.re, b.re};   // Z_0 = A_0 + i B_0
            buf[rix<LOGN>(reg, H)] = {a.im, b.im};   // Z_{N/2}
        } else {
            buf[rix<LOGN>(reg, l)] = {a.re - b.im, a.im + b.re};
            buf[rix<LOGN>(reg, N - l)] = {a.re + b.im, b.re - a.im};
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- row pass, forward
template <typename T, int LOGN, int BC, int EQ, int KIND>
__device__ __forceinline__ void row_forward_pass(SlotRef s, StateRef sst, cplx<T> *buf, double *scratch) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr int R = rows_per_block<T, LOGN, C>();
    constexpr int NREG = C * R / 2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int y0 = tile * R;
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
    double acc[2 * C];
#pragma unroll
    for (int k = 0; k < 2 * C; ++k) acc[k] = 0.0;

    if constexpr (KIND == K_ITER64 || KIND == K_OUTER_UPD || (KIND == K_INNER32 && LOGN >= 12)) {
        // four consecutive points of both rows of a pair per thread: the packed
        // complex value (row 2p + i row 2p+1) goes to LDS in one write.  The FP64
        // iteration (2048^2: 27.7 -> 25.2 us), the mixed outer update, and the FP32
        // inner pass at 4096^2, whose one-row windows re-fetch the stencil rows they
        // share once the rows in flight exceed the L2 (75 -> 71 us); at 2048^2 the
        // FP32 inner pass measured no gain.
#pragma unroll 2
        for (int idx = threadIdx.x; idx < (R / 2) * N / 4; idx += NT) {
            const int p = idx >> (LOGN - 2), x0 = (idx & (N / 4 - 1)) * 4;
            T wv[2][4][C];
            produce_W4x2<T, LOGN, BC, EQ, KIND>(s, sst, y0 + 2 * p, x0, wv, acc);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int pos = (BC == BC_P) ? x0 + k : dct_pos(x0 + k, N);
#pragma unroll
                for (int c = 0; c < C; ++c) buf[rix<LOGN>(c * R / 2 + p, pos)] = cplx<T>{wv[0][k][c], wv[1][k][c]};
            }
        }
    } else {
        // four consecutive points per thread and pass, vector loads
#pragma unroll 2
        for (int idx = threadIdx.x; idx < R * N / 4; idx += NT) {
            const int r = idx >> (LOGN - 2), x0 = (idx & (N / 4 - 1)) * 4;
            T wv[4][C];
            produce_W4<T, LOGN, BC, EQ, KIND>(s, sst, y0 + r, x0, wv, acc);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int pos = (BC == BC_P) ? x0 + k : dct_pos(x0 + k, N);
#pragma unroll
                for (int c = 0; c < C; ++c) rreal<T, LOGN>(buf, c * R / 2 + r / 2, 2 * pos + (r & 1)) = wv[k][c];
            }
        }
    }
    __syncthreads();
    const cplx<T> *twd = (const cplx<T> *)s.twd;
    wg_fft16<T, LOGN, -1, NREG, NT>(buf, twr);
    cplx<T> *S = (cplx<T> *)s.S;
    if constexpr (BC == BC_P) {
        rows_post_store<T, LOGN, C, R, NT>(buf, S, y0);
    } else {
    rows_post_forward<T, LOGN, BC, NREG, NT>(buf, twd);
    // Tile store: this workgroup's R rows are one contiguous block per component;
    // every access of the block is issued before any completes.
    {
        constexpr int SV = spec_vec<T>();
        constexpr int TOT = C * R * H / SV;
#pragma unroll
        for (int i = 0; i < (TOT + NT - 1) / NT; ++i) {
            const int idx = threadIdx.x + i * NT;
            if (TOT % NT == 0 || idx < TOT) {
                const int r0 = (idx % (R / SV)) * SV, rest = idx / (R / SV);
                const int kx = rest % H, c = rest / H;
                cplx<T> v[SV];
#pragma unroll
                for (int q = 0; q < SV; ++q) {
                    const int r = r0 + q;
                    v[q] = buf[rix<LOGN>(c * R / 2 + r / 2, (r & 1) * H + kx)];
                }
                spec_store<T>(&S[spec_off<R>(c, y0 + r0, kx, N)], v);
            }
        }
    }
    }
    write_partials<C>(s, tile, acc, scratch);
}

template <typename T, int LOGN, int BC, int EQ, int KIND>
__global__ __launch_bounds__(NT) void k_row_forward(Slot *const *slots) {
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr int NREG = C * rows_per_block<T, LOGN, C>() / 2;
    __shared__ cplx<T> buf[NREG * lds_region<LOGN>()];
    __shared__ double scratch[2 * C * (NT / 64)];
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if (skip_launch<KIND>(sst)) return;
    if constexpr (KIND == K_MIXED) {
        if (sst.done) row_forward_pass<T, LOGN, BC, EQ, K_OUTER_UPD>(s, sst, buf, scratch);
        else row_forward_pass<T, LOGN, BC, EQ, K_INNER32>(s, sst, buf, scratch);
    } else {
        row_forward_pass<T, LOGN, BC, EQ, KIND>(s, sst, buf, scratch);
    }
}

// ---------------------------------------------------------------- column pass
// A workgroup takes CB adjacent columns of one component, one transform per
// N/16 threads.  CB is chosen so that the CB x R block of a spectrum tile it
// reads is at least 64 bytes (and the workgroup at least one wave), as far as
// 156 KB of LDS (of the 160 KB a gfx950 workgroup may hold) and 1024 threads allow.
// Column blocks are mapped to XCDs in contiguous ranges (xcd_tile), so the two
// blocks that read the halves of a 128-byte line run on the same XCD and the
// second finds it in that XCD's L2.  At 2048^2 this takes the FP32 column pass
// from 4 columns (128-byte runs) and 17.2 us to 2 columns and 15.3 us.
// LDS of one column of a column-pass workgroup: a transform region plus the
// spacing between the regions of the teams of one wave (see cols_regs).
constexpr int COL_TEAM_PAD = 8;
template <int LOGN> constexpr int col_region() { return lds_region<LOGN>() + COL_TEAM_PAD; }

template <typename T, int LOGN, int C> constexpr int col_jobs() {
    constexpr int N = 1 << LOGN;
    constexpr int R = rows_per_block<T, LOGN, C>();
    constexpr int tile_bytes = R * (int)sizeof(cplx<T>);
    constexpr int by_tile = tile_bytes >= 64 ? 1 : 64 / tile_bytes;
    constexpr int by_wave = (N / 16 >= 64) ? 1 : 64 / (N / 16);
    constexpr int want = by_tile > by_wave ? by_tile : by_wave;
    // LDS (<= 156 KB, leaving room for the decision lanes) and threads (<= 1024)
    // bound it from above
    constexpr int by_lds = 159744 / (col_region<LOGN>() * (int)sizeof(cplx<T>));
    constexpr int by_thr = 1024 / (N / 16 >= 1 ? N / 16 : 1);
    constexpr int cap = by_lds < by_thr ? by_lds : by_thr;
    constexpr int cb0 = want < cap ? want : cap;
    constexpr int cb1 = cb0 < 1 ? 1 : (cb0 > N / 2 ? N / 2 : cb0);
    // a power of two, so that it divides N/2
    return cb1 >= 16 ? 16 : cb1 >= 8 ? 8 : cb1 >= 4 ? 4 : cb1 >= 2 ? 2 : 1;
}
template <typename T, int LOGN, int C> constexpr int col_threads() { return col_jobs<T, LOGN, C>() * ((1 << LOGN) / 16); }
// Register budget: two column workgroups must fit on one CU (four SIMDs), so that
// the extra decision workgroup of a launch that fills every CU starts at once --
// where their LDS fits twice in the CU's 160 KB; otherwise one.
template <typename T, int LOGN, int C> constexpr int col_waves_per_eu() {
    constexpr int lds = col_jobs<T, LOGN, C>() * col_region<LOGN>() * (int)sizeof(cplx<T>);
    constexpr int per_cu = 2 * lds + 4096 <= 163840 ? 2 : 1;
    constexpr int w = per_cu * col_threads<T, LOGN, C>() / 64 / 4;
    return w < 1 ? 1 : w;
}

// Periodic column pass with the transforms ended in registers (fft16_regs): each
// thread loads its 16 values of one column straight from S, and the forward
// transform's last pass, the symbol and the inverse transform's first pass run
// on the same registers, so LDS is touched only between passes.  Lanes are laid
// out so that R*CB consecutive lanes read R consecutive rows of the CB columns
// of the block, one contiguous run of the tile layout.  Column 0 of a component
// (which couples bins l and N - l) takes the LDS path instead.  A wave then holds
// several teams, which would hit the same LDS banks at the same offsets of their
// regions: team regions are spaced COL_TEAM_PAD complex values apart beyond the
// region size (64 bytes in FP32: 16 banks).  At N = 2048 the column pass takes
// 21 instead of 26 us (FP64) and 17.1 instead of 18.2 us (FP32).
template <typename T, int LOGN, int C> constexpr bool cols_in_regs() {
    constexpr int TPF = (1 << LOGN) / 16;
    constexpr int R = rows_per_block<T, LOGN, C>();
    return npasses16<LOGN>() >= 2 && TPF >= R && TPF % R == 0;
}

template <typename T, int LOGN, int C, int CB>
__device__ __forceinline__ void cols_regs(SlotRef s, int c, int kx0, cplx<T> *S, cplx<T> *buf) {
    constexpr int N = 1 << LOGN, H = N / 2, TPF = N / 16;
    constexpr int R = rows_per_block<T, LOGN, C>();
    typedef T v2_t __attribute__((ext_vector_type(2)));
    const int idx = threadIdx.x;
    const int team = (idx / R) % CB;
    const int t = (idx / (R * CB)) * R + idx % R;
    const int kx = kx0 + team;
    cplx<T> *x = buf + team * col_region<LOGN>();
    // element t + r N/16 of the column sits r * (N/16) * (N/2) slots after element t
    const int o0 = (int)spec_off<R>(c, t, kx, N);
    constexpr int STRIDE = TPF * H;
    cplx<T> v[16];
    {
        const auto Sg = gp((const v2_t *)S);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const v2_t a = Sg[o0 + r * STRIDE];
            v[r] = {a[0], a[1]};
        }
    }
    {
        Tw16<T, LOGN> twr;
        load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw, t);
        fft16_regs<T, LOGN, -1>(x, t, twr, v);
    }
    {
        const double al = s.alpha[c], be = s.beta[c], ga = s.gamma[c];
        const double invN2 = 1.0 / ((double)N * (double)N);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const T m = (T)symbol_mult(s.eig, kx, t + r * TPF, al, be, ga, invN2);
            v[r] = {v[r].re * m, v[r].im * m};
        }
    }
    __syncthreads();   // the last forward pass has read x
    // gather the twiddles again rather than keeping them live across the symbol,
    // and recompute the LDS addresses of the inverse passes rather than keeping the
    // forward ones (an empty asm hides that t is unchanged; without it the FP32
    // pass spills them)
    __asm__ volatile("" ::: "memory");
    {
        int t2 = t;
        __asm__ volatile("" : "+v"(t2));
        cplx<T> *x2 = buf + ((threadIdx.x / R) % CB) * col_region<LOGN>();
        Tw16<T, LOGN> twr;
        load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw, t2);
        fft16_regs<T, LOGN, +1>(x2, t2, twr, v);
    }
    const auto So = gp((v2_t *)S);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        v2_t a;
        a[0] = v[r].re;
        a[1] = v[r].im;
        So[o0 + r * STRIDE] = a;
    }
}

// FIN >= 0: the launch has one extra workgroup (block 0, dispatched first, so that
// it runs beside the column transforms also when the grid takes more than one
// round of the CUs) that takes the stop decision of the preceding row pass of
// kind FIN.  The other workgroups test the State as it was before that
// decision: a slot that converges at this row pass runs one column pass more,
// whose output nothing reads (the kernels after it see the decision).
constexpr int FIN_NONE = -1;

template <typename T, int LOGN, int BC, int C, int FIN>
__global__ __launch_bounds__((col_threads<T, LOGN, C>()), (col_waves_per_eu<T, LOGN, C>())) void k_cols(Slot *const *slots) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int NTH = col_threads<T, LOGN, C>();
    constexpr int CB = col_jobs<T, LOGN, C>();
    constexpr int R = rows_per_block<T, LOGN, C>();
    __shared__ cplx<T> buf[CB * col_region<LOGN>()];
    __shared__ double lanes[FIN == FIN_NONE ? 1 : 64 * 2 * C];
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if constexpr (FIN != FIN_NONE) {
        if (blockIdx.x == 0) {
            if (!skip_launch<FIN>(sst)) reduce_and_finalize<FIN, C, NTH>(s, lanes);
            return;
        }
    }
    // A column pass transforms unless the step is finished: in the mixed path a
    // pass that starts after the outer update is the first iteration of the next
    // inner loop (outer_done equals done in the FP64 path).
    if (sst.outer_done) return;
    // blockIdx.x -> (component, first column); CB divides N/2
    const int bx = xcd_tile((int)blockIdx.x - (FIN != FIN_NONE ? 1 : 0), C * (H / CB));
    const int c = bx / (H / CB);
    const int kx0 = (bx % (H / CB)) * CB;
    cplx<T> *S = (cplx<T> *)s.S;
    if constexpr (BC == BC_P && cols_in_regs<T, LOGN, C>()) {
        if (kx0 > 0) {
            cols_regs<T, LOGN, C, CB>(s, c, kx0, S, buf);
            return;
        }
    }
    // consecutive threads: rows of a tile, then columns, then tiles; every load of
    // the block is issued before any completes
    constexpr int SV = spec_vec<T>();
    constexpr int TOT = CB * N / SV;
#pragma unroll
    for (int i = 0; i < (TOT + NTH - 1) / NTH; ++i) {
        const int idx = threadIdx.x + i * NTH;
        if (TOT % NTH == 0 || idx < TOT) {
            const int r0 = (idx % (R / SV)) * SV, rest = idx / (R / SV);
            const int reg = rest % CB, yt = rest / CB;
            const int y = yt * R + r0;
            cplx<T> v[SV];
            spec_load<T>(&S[spec_off<R>(c, y, kx0 + reg, N)], v);
#pragma unroll
            for (int q = 0; q < SV; ++q) {
                const int pos = (BC == BC_P) ? y + q : dct_pos(y + q, N);
                buf[rix<LOGN>(reg, pos)] = v[q];
            }
        }
    }
    __syncthreads();
    const cplx<T> *twd = (const cplx<T> *)s.twd;
    {
        Tw16<T, LOGN> twr;
        load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
        wg_fft16<T, LOGN, -1, CB, NTH>(buf, twr);
    }
    cols_apply_symbol<T, LOGN, BC, CB, NTH>(buf, c * H + kx0, CB, s, twd);
    // the inverse transform gathers its twiddles again rather than keeping the
    // forward ones live across the symbol pass (register budget)
    __asm__ volatile("" ::: "memory");
    {
        Tw16<T, LOGN> twr;
        load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
        wg_fft16<T, LOGN, +1, CB, NTH>(buf, twr);
    }
#pragma unroll
    for (int i = 0; i < (TOT + NTH - 1) / NTH; ++i) {
        const int idx = threadIdx.x + i * NTH;
        if (TOT % NTH == 0 || idx < TOT) {
            const int r0 = (idx % (R / SV)) * SV, rest = idx / (R / SV);
            const int reg = rest % CB, yt = rest / CB;
            const int y = yt * R + r0;
            cplx<T> v[SV];
#pragma unroll
            for (int q = 0; q < SV; ++q) {
                const int pos = (BC == BC_P) ? y + q : dct_pos(y + q, N);
                v[q] = buf[rix<LOGN>(reg, pos)];
            }
            spec_store<T>(&S[spec_off<R>(c, y, kx0 + reg, N)], v);
        }
    }
}

// ---------------------------------------------------------------- row pass, inverse + dual update
template <typename T, int LOGN, int BC, int C>
__global__ __launch_bounds__(NT) void k_rowinv(Slot *const *slots) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int R = rows_per_block<T, LOGN, C>();
    constexpr int NREG = C * R / 2;
    __shared__ cplx<T> buf[NREG * lds_region<LOGN>()];
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if (skip_launch<K_ITER64>(sst)) return;
    const int y0 = blockIdx.x * R;
    const size_t NN = (size_t)N * N;
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
    const cplx<T> *S = (const cplx<T> *)s.S;
    const auto P = gp((T *)s.P);
    const auto Pt = gp((T *)s.Pt);
    const bool first = sst.iters == 0;
    // four consecutive points per thread; P_n is loaded before the transforms
    // (when it fits in 64 registers) so that its latency hides behind them
    constexpr int TOTP = C * R * N / 4;
    constexpr int PIT = (TOTP + NT - 1) / NT;
    constexpr bool PREF = PIT * (int)sizeof(T) <= 64;
    vec4_t<T> Pn[PIT];
    auto load_P = [&](int i) {
        const int idx = threadIdx.x + i * NT;
        const int x0 = (idx & (N / 4 - 1)) * 4, rest = idx >> (LOGN - 2);
        const int r = rest % R, c = rest / R;
        if (first) {
#pragma unroll
            for (int k = 0; k < 4; ++k) Pn[i][k] = (T)0;
        } else {
            Pn[i] = load4<T>(P + (c * NN + (size_t)(y0 + r) * N + x0));
        }
    };
    if constexpr (PREF) {
#pragma unroll
        for (int i = 0; i < PIT; ++i)
            if (TOTP % NT == 0 || threadIdx.x + i * NT < TOTP) load_P(i);
    }
    if constexpr (BC == BC_P) {
        rows_load_pre<T, LOGN, C, R, NT>(buf, S, y0);
    } else {
        constexpr int SV = spec_vec<T>();
        constexpr int TOT = C * R * H / SV;
#pragma unroll
        for (int i = 0; i < (TOT + NT - 1) / NT; ++i) {
            const int idx = threadIdx.x + i * NT;
            if (TOT % NT == 0 || idx < TOT) {
                const int r0 = (idx % (R / SV)) * SV, rest = idx / (R / SV);
                const int kx = rest % H, c = rest / H;
                cplx<T> v[SV];
                spec_load<T>(&S[spec_off<R>(c, y0 + r0, kx, N)], v);
#pragma unroll
                for (int q = 0; q < SV; ++q) {
                    const int r = r0 + q;
                    buf[rix<LOGN>(c * R / 2 + r / 2, (r & 1) * H + kx)] = v[q];
                }
            }
        }
        __syncthreads();
        const cplx<T> *twd = (const cplx<T> *)s.twd;
        rows_pre_inverse<T, LOGN, BC, NREG, NT>(buf, twd);
    }
    wg_fft16<T, LOGN, +1, NREG, NT>(buf, twr);
    const T tp = (T)s.tau_p, om = (T)s.omega;
#pragma unroll
    for (int i = 0; i < PIT; ++i) {
        const int idx = threadIdx.x + i * NT;
        if (TOTP % NT != 0 && idx >= TOTP) break;
        const int x0 = (idx & (N / 4 - 1)) * 4, rest = idx >> (LOGN - 2);
        const int r = rest % R, c = rest / R;
        const size_t g = c * NN + (size_t)(y0 + r) * N + x0;
        if constexpr (!PREF) load_P(i);
        vec4_t<T> Pn1, Ptl;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int pos = (BC == BC_P) ? x0 + k : dct_pos(x0 + k, N);
            const cplx<T> zv = buf[rix<LOGN>(c * R / 2 + r / 2, pos)];
            const T Y = (r & 1) ? zv.im : zv.re;
            Pn1[k] = Pn[i][k] + tp * Y;
            Ptl[k] = Pn1[k] + om * (Pn1[k] - Pn[i][k]);
        }
        store4<T>(P + g, Pn1);
        store4<T>(Pt + g, Ptl);
    }
}

// ---------------------------------------------------------------- primal update
// Each thread updates UPD_PPT = 4 consecutive points of one row.
constexpr int UPD_PPT = 4;

template <typename T, int LOGN, int BC, int EQ, int MODE>
__global__ __launch_bounds__(NT) void k_upd(Slot *const *slots) {
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr int N = 1 << LOGN;
    constexpr size_t NN = (size_t)N * N;
    constexpr int HY = stencil_hy<EQ>();
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if (skip_launch<K_ITER64>(sst)) return;
    const size_t g0 = ((size_t)xcd_tile(blockIdx.x, gridDim.x) * NT + threadIdx.x) * UPD_PPT;
    if (g0 >= NN) return;
    const int y = (int)(g0 >> LOGN), x0 = (int)(g0 & (N - 1));
    const int it = sst.iters;
    const auto Pt = gp((const T *)s.Pt);
    const auto Ucur = gp((const T *)s.U[it & 1]);
    const auto Unext = gp((T *)s.U[(it + 1) & 1]);
    Win<T, HY> wp[C];
    vec4_t<T> un[C];
    T Uc[UPD_PPT][C];
    if constexpr (EQ == EQ_FCH) {
        // the FCH adjoint also needs U on the 5-point neighbourhood: the FP64 iterate,
        // or in the mixed inner loop U + e (the FP32 copy of U plus the correction)
        Win<T, 1> wu, we;
        load_win<T, BC, LOGN, HY>(wp[0], Pt, y, x0);
        if constexpr (MODE == MODE_F64) {
            load_win<T, BC, LOGN, 1>(wu, Ucur, y, x0);
            we = wu;
        } else {
            Win<float, 1> wub;
            load_win<float, BC, LOGN, 1>(wub, gp((const float *)s.Ub32), y, x0);
            if (it > 0) load_win<T, BC, LOGN, 1>(we, Ucur, y, x0);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int hx = i == 1 ? 1 : 0;
#pragma unroll
                for (int j = 1 - hx; j < 5 + hx; ++j) {
                    if (it == 0) we.v[i][j] = (T)0;
                    wu.v[i][j] = (T)wub.v[i][j] + we.v[i][j];
                }
            }
        }
        const T tu = (T)s.tau_u;
        vec4_t<T> o;
#pragma unroll
        for (int k = 0; k < UPD_PPT; ++k)
            o[k] = we.at(k, 0, 0) - tu * eval_adjoint_fch<T>(s, [&](int, int dy, int dx) { return wp[0].at(k, dy, dx); },
                                                             [&](int, int dy, int dx) { return wu.at(k, dy, dx); });
        store4<T>(Unext + g0, o);
        return;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        load_win<T, BC, LOGN, HY>(wp[c], Pt + c * NN, y, x0);
        if constexpr (MODE == MODE_F64) {
            un[c] = load4<T>(Ucur + c * NN + g0);
#pragma unroll
            for (int k = 0; k < UPD_PPT; ++k) Uc[k][c] = un[c][k];
        } else {
            // mixed: the iterate is the correction e (e_0 = 0); f' is taken at U + e
            if (it == 0) {
#pragma unroll
                for (int k = 0; k < UPD_PPT; ++k) un[c][k] = (T)0;
            } else {
                un[c] = load4<T>(Ucur + c * NN + g0);
            }
            const vec4_t<float> ub = load4<float>(gp((const float *)s.Ub32) + c * NN + g0);
#pragma unroll
            for (int k = 0; k < UPD_PPT; ++k) Uc[k][c] = (T)ub[k] + un[c][k];
        }
    }
    const T tu = (T)s.tau_u;
    vec4_t<T> out[C];
#pragma unroll
    for (int k = 0; k < UPD_PPT; ++k) {
        T adj[C];
        eval_adjoint<EQ, T>(s, [&](int c, int dy, int dx) { return wp[c].at(k, dy, dx); }, Uc[k], adj);
#pragma unroll
        for (int c = 0; c < C; ++c) out[c][k] = un[c][k] - tu * adj[c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) store4<T>(Unext + c * NN + g0, out[c]);
}

// ---------------------------------------------------------------- kernel-level entry points
// W = F(U) in FP64 with per-workgroup squared-norm partials (no transform).
template <int BC, int EQ>
__global__ __launch_bounds__(NT) void k_residual(const Slot *sp, const double *U, const double *Uk, double *W,
                                                 double *partials) {
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    __shared__ double scratch[C * (NT / 64)];
    SlotRef s = slot_ref(sp);
    const int N = s.N;
    const size_t NN = (size_t)N * N;
    const size_t g = (size_t)blockIdx.x * NT + threadIdx.x;
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    if (g < NN) {
        const int y = (int)(g / N), x = (int)(g % N);
        auto acc_u = [&](int c, int dy, int dx) -> double {
            return U[c * NN + (size_t)wrap<BC>(y + dy, N) * N + wrap<BC>(x + dx, N)];
        };
        double ukc[C], Wv[C], Uc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) ukc[c] = Uk[c * NN + g];
        eval_F<EQ, double>(s, acc_u, ukc, Wv, Uc);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            W[c * NN + g] = Wv[c];
            acc[c] = Wv[c] * Wv[c];
        }
    }
    block_sum<C>(acc, scratch);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) partials[blockIdx.x * C + c] = acc[c];
    }
}

// Pointwise reaction prox of every grid point.
template <int EQ>
__global__ __launch_bounds__(NT) void k_prox(const Slot *sp, const double *cin, double *uout) {
    SlotRef s = slot_ref(sp);
    const size_t NN = (size_t)s.N * s.N;
    const size_t g = (size_t)blockIdx.x * NT + threadIdx.x;
    if (g >= NN) return;
    if constexpr (EQ == EQ_LAP5) {
        uout[g] = prox_ac(cin[g], s.ht, s.b);
    } else if constexpr (EQ == EQ_SCHNAK) {
        double u, v;
        prox_schnak(cin[g], cin[NN + g], s.ht, s.sa, s.sb, s.kappa, u, v);
        uout[g] = u;
        uout[NN + g] = v;
    } else {
        uout[g] = cin[g];
    }
}

// Precondition-only passes (rd_precond_solve): W (FP64) -> row transform -> S,
// then k_cols, then inverse rows -> Y (FP64).  Use the same transform code as the
// iteration; the slot's state is not touched.
template <typename T, int LOGN, int BC, int C>
__global__ __launch_bounds__(NT) void k_rows_transform_in(Slot *const *slots, const double *W) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int R = rows_per_block<T, LOGN, C>();
    constexpr int NREG = C * R / 2;
    __shared__ cplx<T> buf[NREG * lds_region<LOGN>()];
    SlotRef s = slot_of(slots);
    const int y0 = blockIdx.x * R;
    const size_t NN = (size_t)N * N;
#pragma unroll 8
    for (int idx = threadIdx.x; idx < C * R * N; idx += NT) {
        const int x = idx & (N - 1), rest = idx >> LOGN;
        const int r = rest % R, c = rest / R;
        const int pos = (BC == BC_P) ? x : dct_pos(x, N);
        rreal<T, LOGN>(buf, c * R / 2 + r / 2, 2 * pos + (r & 1)) = (T)W[c * NN + (size_t)(y0 + r) * N + x];
    }
    __syncthreads();
    {
        Tw16<T, LOGN> twr;
        load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
        wg_fft16<T, LOGN, -1, NREG, NT>(buf, twr);
    }
    rows_post_forward<T, LOGN, BC, NREG, NT>(buf, (const cplx<T> *)s.twd);
    cplx<T> *S = (cplx<T> *)s.S;
#pragma unroll 8
    for (int idx = threadIdx.x; idx < C * R * H; idx += NT) {
        const int r = idx % R, rest = idx / R;
        const int kx = rest % H, c = rest / H;
        S[spec_off<R>(c, y0 + r, kx, N)] = buf[rix<LOGN>(c * R / 2 + r / 2, (r & 1) * H + kx)];
    }
}

template <typename T, int LOGN, int BC, int C>
__global__ __launch_bounds__(NT) void k_rows_transform_out(Slot *const *slots, double *Y) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int R = rows_per_block<T, LOGN, C>();
    constexpr int NREG = C * R / 2;
    __shared__ cplx<T> buf[NREG * lds_region<LOGN>()];
    SlotRef s = slot_of(slots);
    const int y0 = blockIdx.x * R;
    const size_t NN = (size_t)N * N;
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
    const cplx<T> *S = (const cplx<T> *)s.S;
#pragma unroll 8
    for (int idx = threadIdx.x; idx < C * R * H; idx += NT) {
        const int r = idx % R, rest = idx / R;
        const int kx = rest % H, c = rest / H;
        buf[rix<LOGN>(c * R / 2 + r / 2, (r & 1) * H + kx)] = S[spec_off<R>(c, y0 + r, kx, N)];
    }
    __syncthreads();
    rows_pre_inverse<T, LOGN, BC, NREG, NT>(buf, (const cplx<T> *)s.twd);
    wg_fft16<T, LOGN, +1, NREG, NT>(buf, twr);
#pragma unroll 8
    for (int idx = threadIdx.x; idx < C * R * N; idx += NT) {
        const int x = idx & (N - 1), rest = idx >> LOGN;
        const int r = rest % R, c = rest / R;
        const int pos = (BC == BC_P) ? x : dct_pos(x, N);
        const cplx<T> zv = buf[rix<LOGN>(c * R / 2 + r / 2, pos)];
        Y[c * NN + (size_t)(y0 + r) * N + x] = (double)((r & 1) ? zv.im : zv.re);
    }
}

}  // namespace rdk
