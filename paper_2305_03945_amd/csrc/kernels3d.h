// HIP kernels of the G-prox PDHG iteration on 3-D grids (N^3 points, 7-point
// Laplacian).  The method is posed on a domain in R^d (Sec. 2); with the 7-point
// Laplacian every operator of Algorithm 1 keeps its 2-D form, and G is
// diagonalised by the 3-D DFT (periodic) or DCT-II (Neumann).
//
// Fields are [c][z][y][x], x fastest.  The spectrum S3 holds, for every
// component and (z, y) row, N/2 complex slots, row-major: S3[c][z][y][j].
// One iteration is six launches:
//   k3_rowinv      inverse x-transforms of Y -> P_{n+1}, P~ (eqs. 21-22)
//   k3_upd         U_{n+1} = U_n - tau_u grad F(U_n)^T P~ (eq. 23)
//   k3_row_forward W = F(U_{n+1}) (or F~(e), or the mixed outer update), partial
//                  norms, forward x-transforms
//   k3_lines YFWD  forward y-transforms of the x-spectra; one extra workgroup
//                  takes the stop decision of the preceding row pass
//   k3_lines ZSYM  forward z-transform, multiply by 1 / (N^3 g), inverse z-transform
//   k3_lines YINV  inverse y-transforms
// The x-transform packs two real rows into one complex FFT exactly as the 2-D row
// pass does (rows_post_forward / rows_pre_inverse); the y-pass applies the same
// packing rules to the slot columns that hold real data, so that the z-pass sees,
// per line, either one complex sequence or two real sequences packed as re / im.
#pragma once
#include "kernels.h"

namespace rdk {

// ---------------------------------------------------------------- 3-D stencil windows
// Four consecutive points (z, y, x0 .. x0+3), x0 a multiple of 4, and their 7-point
// neighbourhood: the row (z, y) with one value on each side, and the rows (z, y +- 1)
// and (z +- 1, y) at the four points.
template <typename T> struct Win3 {
    T c[6];        // row (z, y): x0 - 1 .. x0 + 4
    T r[4][4];     // rows (z, y-1), (z, y+1), (z-1, y), (z+1, y): x0 .. x0 + 3
    __device__ __forceinline__ T at(int k, int dz, int dy, int dx) const {
        if (dz == 0 && dy == 0) return c[1 + k + dx];
        if (dz == 0) return r[dy < 0 ? 0 : 1][k];
        return r[dz < 0 ? 2 : 3][k];
    }
};

template <typename T, int BC, int LOGN>
__device__ __forceinline__ void load_win3(Win3<T> &w, gptr_t<const T> f, int z, int y, int x0) {
    constexpr int N = 1 << LOGN;
    const gptr_t<const T> row = f + ((size_t)z * N + y) * N;
    const vec4_t<T> m = load4<T>(row + x0);
#pragma unroll
    for (int k = 0; k < 4; ++k) w.c[1 + k] = m[k];
    w.c[0] = row[wrap<BC>(x0 - 1, N)];
    w.c[5] = row[wrap<BC>(x0 + 4, N)];
    const int ys[4] = {wrap<BC>(y - 1, N), wrap<BC>(y + 1, N), y, y};
    const int zs[4] = {z, z, wrap<BC>(z - 1, N), wrap<BC>(z + 1, N)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const vec4_t<T> v = load4<T>(f + ((size_t)zs[q] * N + ys[q]) * N + x0);
#pragma unroll
        for (int k = 0; k < 4; ++k) w.r[q][k] = v[k];
    }
}

// 7-point Laplacian of component c at the point, from an accessor a(c, dz, dy, dx).
template <typename V, class Acc> __device__ __forceinline__ V lap7_at(Acc a, int c, V ih2) {
    return (a(c, 0, 0, -1) + a(c, 0, 0, 1) + a(c, 0, -1, 0) + a(c, 0, 1, 0) + a(c, -1, 0, 0) + a(c, 1, 0, 0) -
            (V)6 * a(c, 0, 0, 0)) * ih2;
}

// F(U) (eq. 12; Sec. 3.4.1) with the 7-point Laplacian.
template <int EQ, typename V, class Acc>
__device__ __forceinline__ void eval_F3(SlotRef s, Acc u, const V *ukc, V *W, V *Uc) {
    const V ht = (V)s.ht, ih2 = (V)s.inv_h2;
    if constexpr (EQ == EQ_LAP5) {
        const V u0 = u(0, 0, 0, 0);
        const V b = (V)s.b;
        W[0] = u0 - ukc[0] - ht * ((V)s.diff[0] * lap7_at<V>(u, 0, ih2) + b * (u0 - u0 * u0 * u0));
        Uc[0] = u0;
    } else {
        static_assert(EQ == EQ_SCHNAK, "3-D grids: 7-point equations only");
        const V u0 = u(0, 0, 0, 0), v0 = u(1, 0, 0, 0);
        const V kap = (V)s.kappa, u2v = u0 * u0 * v0;
        W[0] = u0 - ukc[0] - ht * ((V)s.diff[0] * lap7_at<V>(u, 0, ih2) + kap * ((V)s.sa - u0 + u2v));
        W[1] = v0 - ukc[1] - ht * ((V)s.diff[1] * lap7_at<V>(u, 1, ih2) + kap * ((V)s.sb - u2v));
        Uc[0] = u0;
        Uc[1] = v0;
    }
}

// F~(e) of the mixed inner loop (the closed-form reaction differences of eval_Ftilde).
template <int EQ, class AccE, class AccU>
__device__ __forceinline__ void eval_Ftilde3(SlotRef s, AccE e, AccU ub, const float *rc, float *W) {
    const float ht = (float)s.ht, ih2 = (float)s.inv_h2;
    if constexpr (EQ == EQ_LAP5) {
        const float e0 = e(0, 0, 0, 0), U = ub(0, 0, 0, 0);
        const float df = (float)s.b * (e0 - 3.0f * U * U * e0 - 3.0f * U * e0 * e0 - e0 * e0 * e0);
        W[0] = rc[0] + e0 - ht * ((float)s.diff[0] * lap7_at<float>(e, 0, ih2) + df);
    } else {
        const float eu0 = e(0, 0, 0, 0), ev0 = e(1, 0, 0, 0);
        const float U = ub(0, 0, 0, 0), Vv = ub(1, 0, 0, 0);
        const float d = 2.0f * U * Vv * eu0 + U * U * ev0 + Vv * eu0 * eu0 + 2.0f * U * eu0 * ev0 + eu0 * eu0 * ev0;
        const float kap = (float)s.kappa;
        W[0] = rc[0] + eu0 - ht * ((float)s.diff[0] * lap7_at<float>(e, 0, ih2) + kap * (-eu0 + d));
        W[1] = rc[1] + ev0 - ht * ((float)s.diff[1] * lap7_at<float>(e, 1, ih2) - kap * d);
    }
}

// grad F(U)^T P~ (eq. 23; Sec. 3.4.1) with the 7-point Laplacian.
template <int EQ, typename V, class Acc>
__device__ __forceinline__ void eval_adjoint3(SlotRef s, Acc p, const V *Uc, V *out) {
    const V ht = (V)s.ht, ih2 = (V)s.inv_h2;
    if constexpr (EQ == EQ_LAP5) {
        const V p0 = p(0, 0, 0, 0), U = Uc[0];
        out[0] = p0 - (V)s.diff[0] * ht * lap7_at<V>(p, 0, ih2) - ht * ((V)s.b * ((V)1 - (V)3 * U * U)) * p0;
    } else {
        const V p0 = p(0, 0, 0, 0), q0 = p(1, 0, 0, 0);
        const V U = Uc[0], Vv = Uc[1], kap = (V)s.kappa;
        out[0] = p0 - ht * ((V)s.diff[0] * lap7_at<V>(p, 0, ih2) + kap * (-p0 + (V)2 * U * Vv * (p0 - q0)));
        out[1] = q0 - ht * ((V)s.diff[1] * lap7_at<V>(p, 1, ih2) + kap * U * U * (p0 - q0));
    }
}

// ---------------------------------------------------------------- row producer (x-pass)
// The row-forward quantity of every kind (as produce_W4) at four consecutive points
// (z, y, x0..x0+3) of a 3-D grid.
template <typename T, int LOGN, int BC, int EQ, int KIND>
__device__ __forceinline__ void produce3_W4(SlotRef s, StateRef sst, int z, int y, int x0,
                                            T (*wv)[EQ == EQ_SCHNAK ? 2 : 1], double *acc) {
    constexpr int N = 1 << LOGN;
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr size_t NN = (size_t)N * N * N;
    const int it = sst.iters;
    const size_t g0 = ((size_t)z * N + y) * N + x0;
    if constexpr (KIND == K_INNER32) {
        const auto E = gp((const float *)s.U[(it + 1) & 1]);
        Win3<float> we[C];
        vec4_t<float> ub[C], r4[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            load_win3<float, BC, LOGN>(we[c], E + c * NN, z, y, x0);
            ub[c] = load4<float>(gp((const float *)s.Ub32) + c * NN + g0);
            r4[c] = load4<float>(gp((const float *)s.r32) + c * NN + g0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float rc[C], W[C];
#pragma unroll
            for (int c = 0; c < C; ++c) rc[c] = r4[c][k];
            eval_Ftilde3<EQ>(s, [&](int c, int dz, int dy, int dx) { return we[c].at(k, dz, dy, dx); },
                             [&](int c, int, int, int) { return ub[c][k]; }, rc, W);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                acc[c] += (double)W[c] * (double)W[c];
                wv[k][c] = (T)W[c];
            }
        }
    } else {
        Win3<double> wu[C];
        vec4_t<double> uk[C];
        if constexpr (KIND == K_ITER64) {
            const auto Un = gp((const double *)s.U[(it + 1) & 1]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                load_win3<double, BC, LOGN>(wu[c], Un + c * NN, z, y, x0);
                uk[c] = load4<double>(gp((const double *)s.Uk) + c * NN + g0);
            }
        } else if constexpr (KIND == K_INIT64 || KIND == K_OUTER_INIT) {
            const auto src = gp(s.src);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                load_win3<double, BC, LOGN>(wu[c], src + c * NN, z, y, x0);
#pragma unroll
                for (int k = 0; k < 4; ++k) uk[c][k] = wu[c].c[1 + k];
            }
            if (s.init != 0) {
                // predictor U_0 = prox(U^k) at every window value
                auto px = [&](double &a, double &b) {
                    if constexpr (EQ == EQ_LAP5) {
                        a = prox_ac(a, s.ht, s.b);
                    } else {
                        double pu, pv;
                        prox_schnak(a, b, s.ht, s.sa, s.sb, s.kappa, pu, pv);
                        a = pu;
                        b = pv;
                    }
                };
                double dummy = 0.0;
#pragma unroll
                for (int j = 0; j < 6; ++j) px(wu[0].c[j], C == 2 ? wu[C - 1].c[j] : dummy);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int k = 0; k < 4; ++k) px(wu[0].r[q][k], C == 2 ? wu[C - 1].r[q][k] : dummy);
            }
        } else {
            const auto Ucur = gp((const double *)s.U64[sst.outer & 1]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                load_win3<double, BC, LOGN>(wu[c], Ucur + c * NN, z, y, x0);
                uk[c] = load4<double>(gp((const double *)s.Uk) + c * NN + g0);
            }
            if (sst.iters > 0) {
                const auto E = gp((const float *)s.U[sst.iters & 1]);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    Win3<float> we;
                    load_win3<float, BC, LOGN>(we, E + c * NN, z, y, x0);
#pragma unroll
                    for (int j = 0; j < 6; ++j) wu[c].c[j] += (double)we.c[j];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int k = 0; k < 4; ++k) wu[c].r[q][k] += (double)we.r[q][k];
                }
            }
        }
        vec4_t<double> Uc4[C], W4[C];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double W[C], Uc[C], ukc[C];
#pragma unroll
            for (int c = 0; c < C; ++c) ukc[c] = uk[c][k];
            eval_F3<EQ, double>(s, [&](int c, int dz, int dy, int dx) { return wu[c].at(k, dz, dy, dx); }, ukc, W,
                                Uc);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                acc[c] += W[c] * W[c];
                acc[C + c] += Uc[c] - ukc[c];
                Uc4[c][k] = Uc[c];
                W4[c][k] = W[c];
                wv[k][c] = (KIND == K_OUTER_INIT || KIND == K_OUTER_UPD) ? (T)(float)W[c] : (T)W[c];
            }
        }
        if constexpr (KIND != K_ITER64) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if constexpr (KIND == K_INIT64) store4<double>(gp((double *)s.U[0]) + c * NN + g0, Uc4[c]);
                else if constexpr (KIND == K_OUTER_INIT) store4<double>(gp(s.U64[0]) + c * NN + g0, Uc4[c]);
                else store4<double>(gp(s.U64[(sst.outer + 1) & 1]) + c * NN + g0, Uc4[c]);
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
    }
}

// Offset of slot j of row (z, y) of component c in S3 (complex units).
template <int LOGN> __device__ __forceinline__ size_t s3_off(int c, int z, int y, int j) {
    constexpr int N = 1 << LOGN;
    return (((size_t)c * N + z) * N + y) * (N / 2) + j;
}

// ---------------------------------------------------------------- x-pass, forward
// Workgroup = R consecutive rows (z, y0 .. y0+R-1) of every component.
template <typename T, int LOGN, int BC, int EQ, int KIND>
__device__ __forceinline__ void row3_forward_pass(SlotRef s, StateRef sst, cplx<T> *buf, double *scratch) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr int R = rows_per_block3<T, LOGN, C>();
    constexpr int NREG = C * R / 2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int z = tile / (N / R), y0 = (tile % (N / R)) * R;
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
    double acc[2 * C];
#pragma unroll
    for (int k = 0; k < 2 * C; ++k) acc[k] = 0.0;
#pragma unroll 2
    for (int idx = threadIdx.x; idx < R * N / 4; idx += NT) {
        const int r = idx >> (LOGN - 2), x0 = (idx & (N / 4 - 1)) * 4;
        T wv[4][C];
        produce3_W4<T, LOGN, BC, EQ, KIND>(s, sst, z, y0 + r, x0, wv, acc);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int pos = (BC == BC_P) ? x0 + k : dct_pos(x0 + k, N);
#pragma unroll
            for (int c = 0; c < C; ++c) rreal<T, LOGN>(buf, c * R / 2 + r / 2, 2 * pos + (r & 1)) = wv[k][c];
        }
    }
    __syncthreads();
    wg_fft16<T, LOGN, -1, NREG, NT>(buf, twr);
    rows_post_forward<T, LOGN, BC, NREG, NT>(buf, (const cplx<T> *)s.twd);
    cplx<T> *S = (cplx<T> *)s.S;
    for (int idx = threadIdx.x; idx < C * R * H; idx += NT) {
        const int j = idx % H, rest = idx / H;
        const int r = rest % R, c = rest / R;
        S[s3_off<LOGN>(c, z, y0 + r, j)] = buf[rix<LOGN>(c * R / 2 + r / 2, (r & 1) * H + j)];
    }
    write_partials<C>(s, tile, acc, scratch);
}

// KIND K_MIXED: the inner FP32 pass or, once the inner loop has stopped, the FP64
// outer update, read from the State (as the 2-D row pass).
template <typename T, int LOGN, int BC, int EQ, int KIND>
__global__ __launch_bounds__(NT) void k3_row_forward(Slot *const *slots) {
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr int NREG = C * rows_per_block3<T, LOGN, C>() / 2;
    __shared__ cplx<T> buf[NREG * lds_region<LOGN>()];
    __shared__ double scratch[2 * C * (NT / 64)];
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if (skip_launch<KIND>(sst)) return;
    if constexpr (KIND == K_MIXED) {
        if (sst.done) row3_forward_pass<T, LOGN, BC, EQ, K_OUTER_UPD>(s, sst, buf, scratch);
        else row3_forward_pass<T, LOGN, BC, EQ, K_INNER32>(s, sst, buf, scratch);
    } else {
        row3_forward_pass<T, LOGN, BC, EQ, KIND>(s, sst, buf, scratch);
    }
}

// ---------------------------------------------------------------- x-pass, inverse + dual update
template <typename T, int LOGN, int BC, int C>
__global__ __launch_bounds__(NT) void k3_rowinv(Slot *const *slots) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int R = rows_per_block3<T, LOGN, C>();
    constexpr int NREG = C * R / 2;
    constexpr size_t NN = (size_t)N * N * N;
    __shared__ cplx<T> buf[NREG * lds_region<LOGN>()];
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if (skip_launch<K_ITER64>(sst)) return;
    const int tile = blockIdx.x;
    const int z = tile / (N / R), y0 = (tile % (N / R)) * R;
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
    const cplx<T> *S = (const cplx<T> *)s.S;
    for (int idx = threadIdx.x; idx < C * R * H; idx += NT) {
        const int j = idx % H, rest = idx / H;
        const int r = rest % R, c = rest / R;
        buf[rix<LOGN>(c * R / 2 + r / 2, (r & 1) * H + j)] = S[s3_off<LOGN>(c, z, y0 + r, j)];
    }
    __syncthreads();
    rows_pre_inverse<T, LOGN, BC, NREG, NT>(buf, (const cplx<T> *)s.twd);
    wg_fft16<T, LOGN, +1, NREG, NT>(buf, twr);
    const auto P = gp((T *)s.P);
    const auto Pt = gp((T *)s.Pt);
    const T tp = (T)s.tau_p, om = (T)s.omega;
    const bool first = sst.iters == 0;
    for (int idx = threadIdx.x; idx < C * R * N / 4; idx += NT) {
        const int x0 = (idx & (N / 4 - 1)) * 4, rest = idx >> (LOGN - 2);
        const int r = rest % R, c = rest / R;
        const size_t g = c * NN + ((size_t)z * N + y0 + r) * N + x0;
        vec4_t<T> Pn;
        if (first) {
#pragma unroll
            for (int k = 0; k < 4; ++k) Pn[k] = (T)0;
        } else {
            Pn = load4<T>(P + g);
        }
        vec4_t<T> Pn1, Ptl;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int pos = (BC == BC_P) ? x0 + k : dct_pos(x0 + k, N);
            const cplx<T> zv = buf[rix<LOGN>(c * R / 2 + r / 2, pos)];
            const T Y = (r & 1) ? zv.im : zv.re;
            Pn1[k] = Pn[k] + tp * Y;
            Ptl[k] = Pn1[k] + om * (Pn1[k] - Pn[k]);
        }
        store4<T>(P + g, Pn1);
        store4<T>(Pt + g, Ptl);
    }
}

// ---------------------------------------------------------------- primal update
// z-planes one thread of the primal update walks (0: one set of four points per
// thread).  Walking in z, the thread keeps P~ of planes z - 1, z, z + 1 at its
// four points in registers, so its z-neighbours need no load: per set of four
// points the thread requests P~ from the caches three times (centre row and
// the rows y - 1, y + 1) instead of five.  The HBM bytes stay the same (the
// counters read 412 MB per launch either way, 403 MB algorithmic); what drops
// is the number of requests the CUs send to L2, and the FP64 update on 256^3
// runs 131 -> 101 us per launch with 32 planes per thread (16: 109, 8: 114).
// FP32 on 256^3 and both precisions on 128^3 measured no gain or a loss, and
// keep one set of points per thread.
template <typename T, int LOGN> constexpr int upd3_zb() { return (sizeof(T) == 8 && LOGN >= 8) ? 32 : 0; }
template <typename T, int LOGN> constexpr int upd3_blocks() {
    constexpr size_t N = (size_t)1 << LOGN;
    return upd3_zb<T, LOGN>() == 0 ? (int)((N * N * N / 4 + NT - 1) / NT)
                                   : (int)(N * N / (4 * NT) * (N / upd3_zb<T, LOGN>()));
}

template <typename T, int LOGN, int BC, int EQ, int MODE>
__global__ __launch_bounds__(NT) void k3_upd(Slot *const *slots) {
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr int N = 1 << LOGN;
    constexpr size_t NN = (size_t)N * N * N;
    constexpr size_t PL = (size_t)N * N;
    constexpr int ZB = upd3_zb<T, LOGN>();
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if (skip_launch<K_ITER64>(sst)) return;
    if constexpr (ZB > 0) {
        // workgroup -> (block of ZB planes, tile of 4 NT points of a plane);
        // consecutive workgroups (one XCD) take adjacent tiles of the same planes
        constexpr int TPP = (int)(PL / (4 * NT));
        const int b = xcd_tile(blockIdx.x, gridDim.x);
        const int z0 = (b / TPP) * ZB;
        const size_t off = ((size_t)(b % TPP) * NT + threadIdx.x) * 4;   // in-plane
        const int x0 = (int)(off & (N - 1)), y = (int)(off >> LOGN);
        const size_t rowm = (size_t)wrap<BC>(y - 1, N) * N + x0, rowp = (size_t)wrap<BC>(y + 1, N) * N + x0;
        const size_t xl = (size_t)y * N + wrap<BC>(x0 - 1, N), xr = (size_t)y * N + wrap<BC>(x0 + 4, N);
        const int it = sst.iters;
        const auto Pt = gp((const T *)s.Pt);
        const auto Ucur = gp((const T *)s.U[it & 1]);
        const auto Unext = gp((T *)s.U[(it + 1) & 1]);
        const auto Ub = gp((const float *)s.Ub32);
        const T tu = (T)s.tau_u;
        vec4_t<T> pm[C], pc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            pm[c] = load4<T>(Pt + c * NN + (size_t)wrap<BC>(z0 - 1, N) * PL + off);
            pc[c] = load4<T>(Pt + c * NN + (size_t)z0 * PL + off);
        }
#pragma unroll 2
        for (int j = 0; j < ZB; ++j) {
            const int z = z0 + j;
            const size_t pz = (size_t)z * PL;
            Win3<T> wp[C];
            vec4_t<T> pn[C], un[C];
            T Uc[4][C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const auto P = Pt + c * NN;
                pn[c] = load4<T>(P + (size_t)wrap<BC>(z + 1, N) * PL + off);
                wp[c].c[0] = P[pz + xl];
                wp[c].c[5] = P[pz + xr];
                const vec4_t<T> ym = load4<T>(P + pz + rowm), yp = load4<T>(P + pz + rowp);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    wp[c].c[1 + k] = pc[c][k];
                    wp[c].r[0][k] = ym[k];
                    wp[c].r[1][k] = yp[k];
                    wp[c].r[2][k] = pm[c][k];
                    wp[c].r[3][k] = pn[c][k];
                }
                if constexpr (MODE == MODE_F64) {
                    un[c] = load4<T>(Ucur + c * NN + pz + off);
#pragma unroll
                    for (int k = 0; k < 4; ++k) Uc[k][c] = un[c][k];
                } else {
                    if (it == 0) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) un[c][k] = (T)0;
                    } else {
                        un[c] = load4<T>(Ucur + c * NN + pz + off);
                    }
                    const vec4_t<float> ub = load4<float>(Ub + c * NN + pz + off);
#pragma unroll
                    for (int k = 0; k < 4; ++k) Uc[k][c] = (T)ub[k] + un[c][k];
                }
            }
            vec4_t<T> out[C];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                T adj[C];
                eval_adjoint3<EQ, T>(s, [&](int c, int dz, int dy, int dx) { return wp[c].at(k, dz, dy, dx); },
                                     Uc[k], adj);
#pragma unroll
                for (int c = 0; c < C; ++c) out[c][k] = un[c][k] - tu * adj[c];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                store4<T>(Unext + c * NN + pz + off, out[c]);
                pm[c] = pc[c];
                pc[c] = pn[c];
            }
        }
        return;
    }
    const size_t g0 = ((size_t)xcd_tile(blockIdx.x, gridDim.x) * NT + threadIdx.x) * 4;
    if (g0 >= NN) return;
    const int x0 = (int)(g0 & (N - 1)), y = (int)((g0 >> LOGN) & (N - 1)), z = (int)(g0 >> (2 * LOGN));
    const int it = sst.iters;
    const auto Pt = gp((const T *)s.Pt);
    const auto Ucur = gp((const T *)s.U[it & 1]);
    const auto Unext = gp((T *)s.U[(it + 1) & 1]);
    Win3<T> wp[C];
    vec4_t<T> un[C];
    T Uc[4][C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        load_win3<T, BC, LOGN>(wp[c], Pt + c * NN, z, y, x0);
        if constexpr (MODE == MODE_F64) {
            un[c] = load4<T>(Ucur + c * NN + g0);
#pragma unroll
            for (int k = 0; k < 4; ++k) Uc[k][c] = un[c][k];
        } else {
            if (it == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k) un[c][k] = (T)0;
            } else {
                un[c] = load4<T>(Ucur + c * NN + g0);
            }
            const vec4_t<float> ub = load4<float>(gp((const float *)s.Ub32) + c * NN + g0);
#pragma unroll
            for (int k = 0; k < 4; ++k) Uc[k][c] = (T)ub[k] + un[c][k];
        }
    }
    const T tu = (T)s.tau_u;
    vec4_t<T> out[C];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T adj[C];
        eval_adjoint3<EQ, T>(s, [&](int c, int dz, int dy, int dx) { return wp[c].at(k, dz, dy, dx); }, Uc[k], adj);
#pragma unroll
        for (int c = 0; c < C; ++c) out[c][k] = un[c][k] - tu * adj[c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) store4<T>(Unext + c * NN + g0, out[c]);
}

// ---------------------------------------------------------------- y and z passes
enum { L3_YFWD = 0, L3_ZSYM = 1, L3_YINV = 2 };

// Adjacent slots per workgroup: 128 contiguous bytes per line position (64 for
// FP32 on 256^3, where the blocks are mapped to XCDs in contiguous ranges, see
// k3_lines).
template <int LOGN> constexpr bool lines_xcd() { return LOGN >= 8; }
template <typename T, int LOGN> constexpr int line_cb() {
    constexpr int want = ((sizeof(T) == 4 && lines_xcd<LOGN>()) ? 64 : 128) / (int)sizeof(cplx<T>);
    return want > (1 << LOGN) / 2 ? (1 << LOGN) / 2 : want;
}
template <typename T, int LOGN> constexpr int line_threads() {
    constexpr int t = line_cb<T, LOGN>() * ((1 << LOGN) / 16);
    return t < 64 ? 64 : t;
}

// Symbol of the 3-D preconditioner: 1 / (N^3 g), mu = s_kx + s_ky + s_kz.
__device__ __forceinline__ double symbol3(const double *__restrict__ eig, int kx, int ky, int kz, double al,
                                          double be, double ga, double invN3) {
    const double mu = eig[kx] + eig[ky] + eig[kz];
    const double a = 1.0 + mu * (al + mu * (be + ga * mu));
    return invN3 / (a * a);
}

// The z-pass between its forward and inverse transforms: multiply every z-line by
// the symbol.  Region reg holds slot j = j0 + reg of the y-transformed row q.
// Periodic: slot j > 0 holds (kx = j, ky = q), one complex sequence.  Slot 0 holds
// the y-pass's split of the packed kx = 0 / kx = N/2 column: q in (0, N/2) is
// (0, q), q in (N/2, N) is (N/2, q - N/2), and q = 0, q = N/2 hold two real
// sequences packed as re / im: (0, 0) / (0, N/2) and (N/2, 0) / (N/2, N/2).
// Neumann: every line holds two real sequences (cosine coefficients), re / im:
// q < N/2: (2j, 2q) / (2j, 2q+1); q >= N/2: (2j+1, 2q') / (2j+1, 2q'+1), q' = q - N/2.
template <typename T, int LOGN, int BC, int NREG, int NTH>
__device__ __forceinline__ void lines_apply_symbol3(cplx<T> *buf, int c, int q, int j0, SlotRef s,
                                                    const cplx<T> *__restrict__ twd) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int IPT = pair_items_per_thread<LOGN, NREG, NTH>();
    const double invN3 = 1.0 / ((double)N * (double)N * (double)N);
    const double al = s.alpha[c], be = s.beta[c], ga = s.gamma[c];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NTH;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        const int j = j0 + reg;
        const int nl = (l == 0) ? H : N - l;
        cplx<T> &zlr = buf[rix<LOGN>(reg, l)];
        cplx<T> &znr = buf[rix<LOGN>(reg, nl)];
        const cplx<T> zl = zlr, zn = znr;
        // (kx, ky) of the re and im sequences; plain: one complex sequence (a only)
        bool plain;
        int kxa, kya, kxb = 0, kyb = 0;
        if constexpr (BC == BC_P) {
            if (j > 0) {
                plain = true;
                kxa = j;
                kya = q;
            } else if (q != 0 && q != H) {
                plain = true;
                kxa = q < H ? 0 : H;
                kya = q < H ? q : q - H;
            } else {
                plain = false;
                kxa = kxb = (q == 0) ? 0 : H;
                kya = 0;
                kyb = H;
            }
        } else {
            plain = false;
            kxa = kxb = q < H ? 2 * j : 2 * j + 1;
            const int qq = q < H ? q : q - H;
            kya = 2 * qq;
            kyb = 2 * qq + 1;
        }
        if constexpr (BC == BC_P) {
            if (plain) {
                const T m1 = (T)symbol3(s.eig, kxa, kya, l, al, be, ga, invN3);
                const T m2 = (T)symbol3(s.eig, kxa, kya, nl, al, be, ga, invN3);
                zlr = {zl.re * m1, zl.im * m1};
                znr = {zn.re * m2, zn.im * m2};
            } else if (l == 0) {
                zlr = {zl.re * (T)symbol3(s.eig, kxa, kya, 0, al, be, ga, invN3),
                       zl.im * (T)symbol3(s.eig, kxb, kyb, 0, al, be, ga, invN3)};
                znr = {zn.re * (T)symbol3(s.eig, kxa, kya, H, al, be, ga, invN3),
                       zn.im * (T)symbol3(s.eig, kxb, kyb, H, al, be, ga, invN3)};
            } else {
                const T ma = (T)symbol3(s.eig, kxa, kya, l, al, be, ga, invN3);
                const T mb = (T)symbol3(s.eig, kxb, kyb, l, al, be, ga, invN3);
                cplx<T> A = {(zl.re + zn.re) * (T)0.5, (zl.im - zn.im) * (T)0.5};
                cplx<T> B = {(zl.im + zn.im) * (T)0.5, (zn.re - zl.re) * (T)0.5};
                A = {A.re * ma, A.im * ma};
                B = {B.re * mb, B.im * mb};
                zlr = {A.re - B.im, A.im + B.re};
                znr = {A.re + B.im, B.re - A.im};
            }
        } else {
            if (l == 0) {
                zlr = {zl.re * (T)symbol3(s.eig, kxa, kya, 0, al, be, ga, invN3),
                       zl.im * (T)symbol3(s.eig, kxb, kyb, 0, al, be, ga, invN3)};
                znr = {zn.re * (T)symbol3(s.eig, kxa, kya, H, al, be, ga, invN3),
                       zn.im * (T)symbol3(s.eig, kxb, kyb, H, al, be, ga, invN3)};
            } else {
                const cplx<T> w = twd[l];
                const cplx<T> A = {(zl.re + zn.re) * (T)0.5, (zl.im - zn.im) * (T)0.5};
                const cplx<T> B = {(zl.im + zn.im) * (T)0.5, (zn.re - zl.re) * (T)0.5};
                const cplx<T> qa = cmul(A, w), qb = cmul(B, w);
                const T xal = qa.re * (T)symbol3(s.eig, kxa, kya, l, al, be, ga, invN3);
                const T xan = -qa.im * (T)symbol3(s.eig, kxa, kya, N - l, al, be, ga, invN3);
                const T xbl = qb.re * (T)symbol3(s.eig, kxb, kyb, l, al, be, ga, invN3);
                const T xbn = -qb.im * (T)symbol3(s.eig, kxb, kyb, N - l, al, be, ga, invN3);
                const cplx<T> wc = cconj(w);
                const cplx<T> va = cmul(wc, cplx<T>{xal, -xan});
                const cplx<T> vb = cmul(wc, cplx<T>{xbl, -xbn});
                zlr = {va.re - vb.im, va.im + vb.re};
                znr = {va.re + vb.im, vb.re - va.im};
            }
        }
    }
    __syncthreads();
}

// Periodic lines of slots j > 0 are plain complex sequences: the y passes are
// bare transforms and the z pass multiplies by the symbol at (kx, ky, kz) =
// (j, q, l).  Their transforms start from and end in registers (fft16_regs):
// thread t of team g holds elements t + r N/16 of the line of slot j0 + g, and
// CB consecutive lanes take the CB adjacent slots (one 128-byte run).  FP64 only,
// as for the 2-D column pass (measured: no gain for FP32).
template <typename T, int LOGN> constexpr bool lines_in_regs() {
    return sizeof(T) == 8 && npasses16<LOGN>() >= 2 &&
           line_threads<T, LOGN>() == line_cb<T, LOGN>() * ((1 << LOGN) / 16);
}

template <typename T, int LOGN, int PASS>
__device__ __forceinline__ void lines_regs(SlotRef s, int c, int w, int j0, cplx<T> *S, cplx<T> *buf) {
    constexpr int N = 1 << LOGN, TPF = N / 16;
    constexpr int CB = line_cb<T, LOGN>();
    typedef T v2_t __attribute__((ext_vector_type(2)));
    const int team = threadIdx.x % CB, t = threadIdx.x / CB;
    const int j = j0 + team;
    cplx<T> *x = buf + team * lds_region<LOGN>();
    // element p of the line: y lines of plane (c, w), or z lines of row w
    auto off = [&](int p) -> int {
        return PASS == L3_ZSYM ? (int)s3_off<LOGN>(c, p, w, j) : (int)s3_off<LOGN>(c, w, p, j);
    };
    cplx<T> v[16];
    {
        const auto Sg = gp((const v2_t *)S);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const v2_t a = Sg[off(t + r * TPF)];
            v[r] = {a[0], a[1]};
        }
    }
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw, t);
    if constexpr (PASS == L3_ZSYM) {
        fft16_regs<T, LOGN, -1>(x, t, twr, v);
        const double invN3 = 1.0 / ((double)N * (double)N * (double)N);
        const double al = s.alpha[c], be = s.beta[c], ga = s.gamma[c];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const T m = (T)symbol3(s.eig, j, w, t + r * TPF, al, be, ga, invN3);
            v[r] = {v[r].re * m, v[r].im * m};
        }
        __syncthreads();   // the last forward pass has read x
        fft16_regs<T, LOGN, +1>(x, t, twr, v);
    } else {
        fft16_regs<T, LOGN, PASS == L3_YFWD ? -1 : +1>(x, t, twr, v);
    }
    const auto So = gp((v2_t *)S);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        v2_t a;
        a[0] = v[r].re;
        a[1] = v[r].im;
        So[off(t + r * TPF)] = a;
    }
}

// Lines of CB adjacent slots.  YFWD / YINV: the lines along y of plane (c, z);
// ZSYM: the lines along z of row q (the y-transformed index) of component c.
// FIN >= 0 (forward y pass only): one extra workgroup, block 0, takes the stop
// decision of the preceding row pass of kind FIN, as in the 2-D column pass.
template <typename T, int LOGN, int BC, int C, int PASS, int FIN>
__global__ __launch_bounds__((line_threads<T, LOGN>())) void k3_lines(Slot *const *slots) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int CB = line_cb<T, LOGN>();
    constexpr int NTH = line_threads<T, LOGN>();
    static_assert(FIN == FIN_NONE || PASS == L3_YFWD, "only the forward y pass takes a decision");
    __shared__ cplx<T> buf[CB * lds_region<LOGN>()];
    __shared__ double lanes[FIN == FIN_NONE ? 1 : 64 * 2 * C];
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if constexpr (FIN != FIN_NONE) {
        if (blockIdx.x == 0) {
            if (!skip_launch<FIN>(sst)) reduce_and_finalize<FIN, C, NTH>(s, lanes);
            return;
        }
    }
    // The forward y pass transforms unless the step is finished (after a mixed
    // outer update it is the first iteration of the next inner loop, while its
    // decision workgroup runs); the later line passes see a decided State.
    if (PASS == L3_YFWD ? sst.outer_done != 0 : sst.done != 0) return;
    // blockIdx.x -> (component, plane or row, first slot); CB divides N/2
    // 256^3: consecutive blocks (adjacent slot groups, then lines) on one XCD
    // (FP64 line passes 20-25 % faster there; at 128^3 the round-robin order is
    // faster)
    const int b0 = (int)blockIdx.x - (FIN != FIN_NONE ? 1 : 0);
    const int bxl = lines_xcd<LOGN>() ? xcd_tile(b0, C * N * (H / CB)) : b0;
    const int grp = bxl % (H / CB), rest = bxl / (H / CB);
    const int w = rest % N, c = rest / N;
    const int j0 = grp * CB;
    cplx<T> *S = (cplx<T> *)s.S;
    if constexpr (BC == BC_P && lines_in_regs<T, LOGN>()) {
        if (j0 > 0) {
            lines_regs<T, LOGN, PASS>(s, c, w, j0, S, buf);
            return;
        }
    }
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
    // element p of the line of slot j
    auto off = [&](int p, int j) -> size_t {
        return PASS == L3_ZSYM ? s3_off<LOGN>(c, p, w, j) : s3_off<LOGN>(c, w, p, j);
    };
    // in transform order: Makhoul positions for the forward DCT and the final store
    for (int idx = threadIdx.x; idx < CB * N; idx += NTH) {
        const int reg = idx % CB, p = idx / CB;
        const int pos = (PASS == L3_YINV || BC == BC_P) ? p : dct_pos(p, N);
        buf[rix<LOGN>(reg, pos)] = S[off(p, j0 + reg)];
    }
    __syncthreads();
    const cplx<T> *twd = (const cplx<T> *)s.twd;
    if constexpr (PASS == L3_YFWD) {
        wg_fft16<T, LOGN, -1, CB, NTH>(buf, twr);
        // periodic: only slot 0 holds two real sequences (kx = 0 and kx = N/2)
        if constexpr (BC == BC_N) rows_post_forward<T, LOGN, BC, CB, NTH>(buf, twd);
        else if (j0 == 0) rows_post_forward<T, LOGN, BC, 1, NTH>(buf, twd);
    } else if constexpr (PASS == L3_ZSYM) {
        wg_fft16<T, LOGN, -1, CB, NTH>(buf, twr);
        lines_apply_symbol3<T, LOGN, BC, CB, NTH>(buf, c, w, j0, s, twd);
        wg_fft16<T, LOGN, +1, CB, NTH>(buf, twr);
    } else {
        if constexpr (BC == BC_N) rows_pre_inverse<T, LOGN, BC, CB, NTH>(buf, twd);
        else if (j0 == 0) rows_pre_inverse<T, LOGN, BC, 1, NTH>(buf, twd);
        wg_fft16<T, LOGN, +1, CB, NTH>(buf, twr);
    }
    for (int idx = threadIdx.x; idx < CB * N; idx += NTH) {
        const int reg = idx % CB, p = idx / CB;
        const int pos = (PASS == L3_YFWD || BC == BC_P) ? p : dct_pos(p, N);
        S[off(p, j0 + reg)] = buf[rix<LOGN>(reg, pos)];
    }
}

// ---------------------------------------------------------------- preconditioner-only x-passes
template <typename T, int LOGN, int BC, int C>
__global__ __launch_bounds__(NT) void k3_rows_transform_in(Slot *const *slots, const double *W) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int R = rows_per_block3<T, LOGN, C>();
    constexpr int NREG = C * R / 2;
    constexpr size_t NN = (size_t)N * N * N;
    __shared__ cplx<T> buf[NREG * lds_region<LOGN>()];
    SlotRef s = slot_of(slots);
    const int z = blockIdx.x / (N / R), y0 = (blockIdx.x % (N / R)) * R;
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
    for (int idx = threadIdx.x; idx < C * R * N; idx += NT) {
        const int x = idx & (N - 1), rest = idx >> LOGN;
        const int r = rest % R, c = rest / R;
        const int pos = (BC == BC_P) ? x : dct_pos(x, N);
        rreal<T, LOGN>(buf, c * R / 2 + r / 2, 2 * pos + (r & 1)) = (T)W[c * NN + ((size_t)z * N + y0 + r) * N + x];
    }
    __syncthreads();
    wg_fft16<T, LOGN, -1, NREG, NT>(buf, twr);
    rows_post_forward<T, LOGN, BC, NREG, NT>(buf, (const cplx<T> *)s.twd);
    cplx<T> *S = (cplx<T> *)s.S;
    for (int idx = threadIdx.x; idx < C * R * H; idx += NT) {
        const int j = idx % H, rest = idx / H;
        const int r = rest % R, c = rest / R;
        S[s3_off<LOGN>(c, z, y0 + r, j)] = buf[rix<LOGN>(c * R / 2 + r / 2, (r & 1) * H + j)];
    }
}

template <typename T, int LOGN, int BC, int C>
__global__ __launch_bounds__(NT) void k3_rows_transform_out(Slot *const *slots, double *Y) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int R = rows_per_block3<T, LOGN, C>();
    constexpr int NREG = C * R / 2;
    constexpr size_t NN = (size_t)N * N * N;
    __shared__ cplx<T> buf[NREG * lds_region<LOGN>()];
    SlotRef s = slot_of(slots);
    const int z = blockIdx.x / (N / R), y0 = (blockIdx.x % (N / R)) * R;
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
    const cplx<T> *S = (const cplx<T> *)s.S;
    for (int idx = threadIdx.x; idx < C * R * H; idx += NT) {
        const int j = idx % H, rest = idx / H;
        const int r = rest % R, c = rest / R;
        buf[rix<LOGN>(c * R / 2 + r / 2, (r & 1) * H + j)] = S[s3_off<LOGN>(c, z, y0 + r, j)];
    }
    __syncthreads();
    rows_pre_inverse<T, LOGN, BC, NREG, NT>(buf, (const cplx<T> *)s.twd);
    wg_fft16<T, LOGN, +1, NREG, NT>(buf, twr);
    for (int idx = threadIdx.x; idx < C * R * N; idx += NT) {
        const int x = idx & (N - 1), rest = idx >> LOGN;
        const int r = rest % R, c = rest / R;
        const int pos = (BC == BC_P) ? x : dct_pos(x, N);
        const cplx<T> zv = buf[rix<LOGN>(c * R / 2 + r / 2, pos)];
        Y[c * NN + ((size_t)z * N + y0 + r) * N + x] = (double)((r & 1) ? zv.im : zv.re);
    }
}

}  // namespace rdk
