// Small grids: one workgroup runs a whole implicit step.
//
// On N <= 128 grids an iteration moves a few hundred KB, and the four launches of
// the batched iteration (column pass, inverse rows, primal update, forward rows)
// cost their launch latency, not their bytes.  Here one workgroup per slot takes
// the whole step, Algorithm 1 with its stop test, in one launch:
//
//   W = F(U_n) (stencil)  -> spectrum S in LDS (row pairs packed as complex rows)
//   ||W / h_t|| (fixed-order workgroup sum), stop decision (decide<>, thread 0)
//   row FFTs, transpose to columns, column FFTs, 1 / (N^2 g), inverse column
//   FFTs, transpose back, inverse row FFTs          -> Y = G^-1 W_n in LDS
//   P_{n+1} = P_n + tau_p Y,  P~ = P_{n+1} + omega tau_p Y (P~ kept in LDS)
//   U_{n+1} = U_n - tau_u grad F(U_n)^T P~
//
// and, in the mixed precision, the same FP32 inner loop on the correction e with
// the FP64 outer passes (U += e, r = F(U), stop test) between inner loops.  The
// spectrum always lives in LDS; the iterate, P and (mixed) the FP32 copies of U
// and r take LDS in that order while the 160 KB of a gfx950 workgroup allow, and
// otherwise stay in the slot's HBM buffers (then L2-resident).  The arithmetic
// per point is that of the batched kernels (the same eval_F / eval_Ftilde /
// eval_adjoint / transform code); only the order of the norm's sums differs.
#pragma once
#include "kernels.h"

namespace rdk {

constexpr int NT7 = 512;                // threads of a step workgroup
constexpr size_t WG_LDS_BYTES = 163840; // LDS of one gfx950 workgroup

// Which fields of a step fit in LDS beside the spectrum.
template <typename T, int LOGN, int C> struct WgPlan {
    static constexpr int N = 1 << LOGN;
    static constexpr size_t NN = (size_t)N * N;
    static constexpr size_t spec = (size_t)C * (N / 2) * lds_region<LOGN>() * sizeof(cplx<T>);
    static constexpr size_t fixed = 4096;                      // sums, State, tables
    static constexpr size_t fieldT = (size_t)C * NN * sizeof(T);
    static constexpr size_t field32 = (size_t)C * NN * sizeof(float);
    static constexpr size_t room = WG_LDS_BYTES - fixed;
    static constexpr bool ok = spec <= room;
    static constexpr bool u_lds = ok && spec + fieldT <= room;
    static constexpr bool p_lds = u_lds && spec + 2 * fieldT <= room;
    static constexpr bool ub_lds = sizeof(T) == 4 && p_lds && spec + 2 * fieldT + field32 <= room;
    static constexpr bool r_lds = ub_lds && spec + 2 * fieldT + 2 * field32 <= room;
    // FP64 path: U^k as well, when it fits beside U and P
    static constexpr size_t field64 = (size_t)C * NN * sizeof(double);
    static constexpr bool uk_lds = sizeof(T) == 8 && p_lds && spec + 2 * fieldT + field64 <= room;
    static constexpr size_t bytes = spec + (u_lds ? fieldT : 0) + (p_lds ? fieldT : 0) + (ub_lds ? field32 : 0) +
                                    (r_lds ? field32 : 0) + (uk_lds ? field64 : 0);
};

// Whether the single-workgroup step serves (T, N, equation): N <= 64, the
// spectrum fits, and an adjoint that reads U only at its own point (the
// update is made in place), which excludes the sixth-order equation.  (At 128^2
// the fields leave LDS for L2 and the kernel runs out of registers; there the
// batched kernels are faster.)
constexpr int WG_MAX_LOGN = 6;
template <typename T, int LOGN, int EQ> constexpr bool wg_step_available() {
    return LOGN <= WG_MAX_LOGN && EQ != EQ_FCH && WgPlan<T, LOGN, EQ == EQ_SCHNAK ? 2 : 1>::ok;
}

// Workgroup sum of K values per thread in a fixed order (wave butterflies, then
// the waves in order); the totals are valid in thread 0.  red: K * NT7/64 doubles.
template <int K> __device__ __forceinline__ void wg_sum(double *v, double *red) {
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
        for (int k = 0; k < K; ++k) red[k * (NT7 / 64) + wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double x = 0.0;
            for (int w = 0; w < NT7 / 64; ++w) x += red[k * (NT7 / 64) + w];
            v[k] = x;
        }
    }
}

// ---------------------------------------------------------------- column transforms in place
// The column transforms run on the spectrum where the row pass left it (row pairs
// packed per LDS region): element i of column job reg (component c = reg / H,
// column kx = reg % H) is row y of that column, y = i on periodic grids and the
// row whose Makhoul position is i on Neumann grids, at slot (y & 1) H + kx of
// region c H + y / 2.  The Stockham passes of fft16.h with that address map, so
// no transpose is needed between the row and the column transforms.
template <int LOGN, int BC> struct ColMap {
    static constexpr int N = 1 << LOGN, H = N / 2;
    __device__ __forceinline__ static int row_of(int i) {
        if (BC == BC_P) return i;
        return i < H ? 2 * i : 2 * (N - 1 - i) + 1;   // inverse of dct_pos
    }
    __device__ __forceinline__ static int at(int reg, int i) {
        const int c = reg / H, kx = reg % H, y = row_of(i);
        return rix<LOGN>(c * H + (y >> 1), (y & 1) * H + kx);
    }
};

template <typename T, int LOGN, int R, int NS, int DIR, class M>
__device__ __forceinline__ void mpass16(cplx<T> *buf, int reg, int t, bool active, const cplx<T> (*pw)[4]) {
    constexpr int N = 1 << LOGN;
    constexpr int TPF = N / 16;
    constexpr int NB = N / R;
    constexpr int BPT = 16 / R;
    cplx<T> v[BPT][R];
    if (active) {
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int j = t + b * TPF;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = buf[M::at(reg, j + r * NB)];
            if constexpr (NS > 1) {
                cplx<T> p[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if ((1 << e) < R) {
                        p[e] = pw[b][e];
                        if constexpr (DIR > 0) p[e].im = -p[e].im;
                    }
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cplx<T> w = {(T)1, (T)0};
                    bool first = true;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (r & (1 << e)) {
                            w = first ? p[e] : cmul(w, p[e]);
                            first = false;
                        }
                    v[b][r] = cmul(v[b][r], w);
                }
            }
            dftR<T, R, DIR>(v[b]);
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int j = t + b * TPF;
            const int k = j & (NS - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[M::at(reg, base + q * NS)] = v[b][q];
        }
    }
    __syncthreads();
}

template <typename T, int LOGN, int DIR, int DONE, class M>
__device__ __forceinline__ void mpasses16(cplx<T> *buf, int reg, int t, bool active, const Tw16<T, LOGN> &w) {
    if constexpr (DONE < LOGN) {
        constexpr int REM = LOGN - DONE;
        constexpr int R = REM >= 4 ? 16 : (1 << REM);
        constexpr int LOGR = REM >= 4 ? 4 : REM;
        constexpr int q = DONE / 4;
        mpass16<T, LOGN, R, (1 << DONE), DIR, M>(buf, reg, t, active, w.p[q > 0 ? q - 1 : 0]);
        mpasses16<T, LOGN, DIR, DONE + LOGR, M>(buf, reg, t, active, w);
    }
}

// In-place transforms of NREG mapped regions by NTH threads (teams of N/16 take
// regions round-robin); ends with a barrier.
template <typename T, int LOGN, int DIR, int NREG, int NTH, class M>
__device__ __forceinline__ void wg_fft16_mapped(cplx<T> *buf, const Tw16<T, LOGN> &w) {
    constexpr int TPF = (1 << LOGN) / 16;
    constexpr int NTEAMS = NTH / TPF;
    const int team = threadIdx.x / TPF, t = threadIdx.x % TPF;
#pragma unroll 1
    for (int g = 0; g < NREG; g += NTEAMS) {
        const int reg = g + team;
        const bool active = reg < NREG;
        mpasses16<T, LOGN, DIR, 0, M>(buf, active ? reg : 0, t, active, w);
    }
}

// 1 / (N^2 g) on the transformed columns (cols_apply_symbol of fft.h on the
// mapped layout): column job reg of component c = reg / H is kx = reg % H
// (periodic; column 0 packs kx = 0 and kx = N/2) or the cosine pair kx = 2j, 2j + 1
// (Neumann).
template <typename T, int LOGN, int BC, int NREG, int NTH, class M>
__device__ __forceinline__ void cols_symbol_mapped(cplx<T> *buf, SlotRef s, const double *eig, const cplx<T> *twd) {
    constexpr int N = 1 << LOGN, H = N / 2;
    const double invN2 = 1.0 / ((double)N * (double)N);
#pragma unroll 1
    for (int it = threadIdx.x; it < NREG * H; it += NTH) {
        const int reg = it / H, l = it % H;
        const int c = reg / H, j = reg % H;
        const double al = s.alpha[c], be = s.beta[c], ga = s.gamma[c];
        const int nl = (l == 0) ? H : N - l;
        cplx<T> &zlr = buf[M::at(reg, l)];
        cplx<T> &znr = buf[M::at(reg, nl)];
        const cplx<T> zl = zlr, zn = znr;
        if constexpr (BC == BC_P) {
            if (j > 0) {
                const T m1 = (T)symbol_mult(eig, j, l, al, be, ga, invN2);
                const T m2 = (T)symbol_mult(eig, j, nl, al, be, ga, invN2);
                zlr = {zl.re * m1, zl.im * m1};
                znr = {zn.re * m2, zn.im * m2};
            } else if (l == 0) {
                zlr = {zl.re * (T)symbol_mult(eig, 0, 0, al, be, ga, invN2),
                       zl.im * (T)symbol_mult(eig, H, 0, al, be, ga, invN2)};
                znr = {zn.re * (T)symbol_mult(eig, 0, H, al, be, ga, invN2),
                       zn.im * (T)symbol_mult(eig, H, H, al, be, ga, invN2)};
            } else {
                const T ma = (T)symbol_mult(eig, 0, l, al, be, ga, invN2);
                const T mb = (T)symbol_mult(eig, H, l, al, be, ga, invN2);
                cplx<T> A = {(zl.re + zn.re) * (T)0.5, (zl.im - zn.im) * (T)0.5};
                cplx<T> B = {(zl.im + zn.im) * (T)0.5, (zn.re - zl.re) * (T)0.5};
                A = {A.re * ma, A.im * ma};
                B = {B.re * mb, B.im * mb};
                zlr = {A.re - B.im, A.im + B.re};
                znr = {A.re + B.im, B.re - A.im};
            }
        } else {
            const int ka = 2 * j, kb = 2 * j + 1;
            if (l == 0) {
                zlr = {zl.re * (T)symbol_mult(eig, ka, 0, al, be, ga, invN2),
                       zl.im * (T)symbol_mult(eig, kb, 0, al, be, ga, invN2)};
                znr = {zn.re * (T)symbol_mult(eig, ka, H, al, be, ga, invN2),
                       zn.im * (T)symbol_mult(eig, kb, H, al, be, ga, invN2)};
            } else {
                const cplx<T> w = twd[l];
                const cplx<T> A = {(zl.re + zn.re) * (T)0.5, (zl.im - zn.im) * (T)0.5};
                const cplx<T> B = {(zl.im + zn.im) * (T)0.5, (zn.re - zl.re) * (T)0.5};
                const cplx<T> qa = cmul(A, w), qb = cmul(B, w);
                const T xal = qa.re * (T)symbol_mult(eig, ka, l, al, be, ga, invN2);
                const T xan = -qa.im * (T)symbol_mult(eig, ka, N - l, al, be, ga, invN2);
                const T xbl = qb.re * (T)symbol_mult(eig, kb, l, al, be, ga, invN2);
                const T xbn = -qb.im * (T)symbol_mult(eig, kb, N - l, al, be, ga, invN2);
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

// Stencil offsets of reach HY (0: the point; 1: the 5-point stencil; 2: the
// 13-point one) and the slot of (dy, dx) in that list: the point phases gather a
// chunk of points' neighbourhoods into registers before they compute and store, so
// that their loads are not held behind stores to memory they might alias.
template <int HY> struct Stencil {
    static constexpr int NS = HY == 0 ? 1 : (HY == 1 ? 5 : 13);
    __device__ __forceinline__ static constexpr int dy(int i) {
        constexpr int t[13] = {0, 0, 0, -1, 1, -1, -1, 1, 1, 0, 0, -2, 2};
        return t[i];
    }
    __device__ __forceinline__ static constexpr int dx(int i) {
        constexpr int t[13] = {0, -1, 1, 0, 0, -1, 1, -1, 1, -2, 2, 0, 0};
        return t[i];
    }
    __device__ __forceinline__ static constexpr int idx(int y, int x) {
        for (int i = 0; i < 13; ++i)
            if (dy(i) == y && dx(i) == x) return i;
        return 0;
    }
};

// Points per thread, and per chunk of a point phase gathering G values of B bytes
// per point (about 160 bytes of gathered values per thread, within the register
// budget of a 512-thread workgroup).
template <int LOGN> constexpr int wg_ppt() { return (1 << (2 * LOGN)) >= NT7 ? (1 << (2 * LOGN)) / NT7 : 1; }
template <int LOGN, int G, int B> constexpr int wg_chunk() {
    constexpr int c = 160 / (G * B) < 1 ? 1 : 160 / (G * B);
    constexpr int ppt = wg_ppt<LOGN>();
    return c >= ppt ? ppt : (c >= 8 ? 8 : c >= 4 ? 4 : c >= 2 ? 2 : 1);
}

template <typename T, int LOGN, int BC, int EQ, int MODE>
__global__ __launch_bounds__(NT7) void k_step_wg(Slot *const *slots) {
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int NN = N * N;
    constexpr int NREG = C * H;   // row-pair regions = column regions
    constexpr int HY = stencil_hy<EQ>();
    constexpr int HU = EQ == EQ_BIH ? 1 : 0;   // reach of U in the mixed inner residual
    using SY = Stencil<HY>;
    using SU = Stencil<HU>;
    constexpr int PPT = wg_ppt<LOGN>();
    using Plan = WgPlan<T, LOGN, C>;
    static_assert(Plan::ok, "the spectrum must fit in LDS");
    static_assert(MODE == MODE_F64 ? sizeof(T) == 8 : sizeof(T) == 4, "FP64 step or FP32 inner loop");
    __shared__ __align__(16) unsigned char lds[Plan::bytes];
    __shared__ double red[2 * C * (NT7 / 64)];
    __shared__ State stl;
    __shared__ double eig_l[N];        // s_k, and the DCT twiddles: read in LDS phases,
    __shared__ cplx<T> twd_l[N];       // so staged once rather than fetched from L2

    SlotRef s = slot_of(slots);
    const int tid = threadIdx.x;
    cplx<T> *S = (cplx<T> *)lds;
    unsigned char *nxt = lds + Plan::spec;
    // iterate: FP64 U, or the mixed path's correction e
    T *U = Plan::u_lds ? (T *)nxt : (T *)s.U[0];
    nxt += Plan::u_lds ? Plan::fieldT : 0;
    T *P = Plan::p_lds ? (T *)nxt : (T *)s.P;
    nxt += Plan::p_lds ? Plan::fieldT : 0;
    float *Ub = Plan::ub_lds ? (float *)nxt : s.Ub32;
    nxt += Plan::ub_lds ? Plan::field32 : 0;
    float *Rr = Plan::r_lds ? (float *)nxt : s.r32;
    nxt += Plan::r_lds ? Plan::field32 : 0;
    const double *src = s.src;     // U^k: the caller's input, read-only for the whole step
    const double *Ukp = Plan::uk_lds ? (const double *)nxt : src;
    double *U64 = s.U64[0];        // mixed: FP64 U (never bound to the caller's input)
    Tw16<T, LOGN> twr;
    load_tw16<T, LOGN>(twr, (const cplx<T> *)s.tw);
    const StopRule rule{s.tol, s.inner_rtol, s.max_iter, s.max_outer};
    auto pos = [](int x) { return BC == BC_P ? x : dct_pos(x, N); };
    auto at = [](int c, int y, int x) { return c * NN + wrap<BC>(y, N) * N + wrap<BC>(x, N); };
    auto pt_of = [&](int i) { return tid + i * NT7; };
    if (tid == 0) stl = State{};
    for (int i = tid; i < N; i += NT7) {
        eig_l[i] = s.eig[i];
        twd_l[i] = ((const cplx<T> *)s.twd)[i];
    }
    if constexpr (Plan::uk_lds)
        for (int g = tid; g < C * NN; g += NT7) ((double *)Ukp)[g] = src[g];
    const cplx<T> *twd = twd_l;

    // ---- the residual of an FP64 state (U_0, or the mixed outer U) into S; its
    // norm and sum(U - U^k) decided by thread 0
    auto residual64 = [&](const double *Uf, auto decide_fn) {
        constexpr int CK = wg_chunk<LOGN, C *(SY::NS + 1), 8>();
        double acc[2 * C];
#pragma unroll
        for (int k = 0; k < 2 * C; ++k) acc[k] = 0.0;
#pragma unroll 1
        for (int i0 = 0; i0 < PPT; i0 += CK) {
            double v[CK][C][SY::NS], uk[CK][C];
#pragma unroll
            for (int j = 0; j < CK; ++j) {
                const int g = pt_of(i0 + j);
                if (g >= NN) continue;
                const int y = g >> LOGN, x = g & (N - 1);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    uk[j][c] = Ukp[c * NN + g];
#pragma unroll
                    for (int q = 0; q < SY::NS; ++q) v[j][c][q] = Uf[at(c, y + SY::dy(q), x + SY::dx(q))];
                }
            }
#pragma unroll
            for (int j = 0; j < CK; ++j) {
                const int g = pt_of(i0 + j);
                if (g >= NN) continue;
                const int y = g >> LOGN, x = g & (N - 1);
                double W[C], Uc[C];
                eval_F<EQ, double>(s, [&](int c, int dy, int dx) { return v[j][c][SY::idx(dy, dx)]; }, uk[j], W, Uc);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    acc[c] += W[c] * W[c];
                    acc[C + c] += Uc[c] - uk[j][c];
                    if constexpr (MODE == MODE_MIXED) {
                        Rr[c * NN + g] = (float)W[c];
                        Ub[c * NN + g] = (float)Uc[c];
                    }
                    rreal<T, LOGN>(S, c * H + y / 2, 2 * pos(x) + (y & 1)) = (T)W[c];
                }
            }
        }
        wg_sum<2 * C>(acc, red);
        if (tid == 0) {
            double res = 0.0, m = 0.0;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                res += sqrt(acc[c]);
                m += acc[C + c];
            }
            decide_fn(res / s.ht, m);
        }
        __syncthreads();
    };

    // ---- the mixed inner residual F~(e) into S; its norm decided by thread 0
    auto residual32 = [&]() {
        constexpr int CK = wg_chunk<LOGN, C *(SY::NS + SU::NS + 1), 4>();
        double acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0.0;
#pragma unroll 1
        for (int i0 = 0; i0 < PPT; i0 += CK) {
            float ve[CK][C][SY::NS], vu[CK][C][SU::NS], rc[CK][C];
#pragma unroll
            for (int j = 0; j < CK; ++j) {
                const int g = pt_of(i0 + j);
                if (g >= NN) continue;
                const int y = g >> LOGN, x = g & (N - 1);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    rc[j][c] = Rr[c * NN + g];
#pragma unroll
                    for (int q = 0; q < SY::NS; ++q) ve[j][c][q] = (float)U[at(c, y + SY::dy(q), x + SY::dx(q))];
#pragma unroll
                    for (int q = 0; q < SU::NS; ++q) vu[j][c][q] = Ub[at(c, y + SU::dy(q), x + SU::dx(q))];
                }
            }
#pragma unroll
            for (int j = 0; j < CK; ++j) {
                const int g = pt_of(i0 + j);
                if (g >= NN) continue;
                const int y = g >> LOGN, x = g & (N - 1);
                float W[C];
                eval_Ftilde<EQ>(s, [&](int c, int dy, int dx) { return ve[j][c][SY::idx(dy, dx)]; },
                                [&](int c, int dy, int dx) { return vu[j][c][SU::idx(dy, dx)]; }, rc[j], W);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    acc[c] += (double)W[c] * (double)W[c];
                    rreal<T, LOGN>(S, c * H + y / 2, 2 * pos(x) + (y & 1)) = (T)W[c];
                }
            }
        }
        wg_sum<C>(acc, red);
        if (tid == 0) {
            double res = 0.0;
#pragma unroll
            for (int c = 0; c < C; ++c) res += sqrt(acc[c]);
            stl = decide<K_INNER32>(stl, rule, res / s.ht, 0.0);
        }
        __syncthreads();
    };

    // ---- Y = G^-1 W in place (W in S as packed row pairs on entry; on exit the
    // complex slot pos(x) of region c H + y / 2 holds Y of rows y, y + 1 as re, im)
    auto precond = [&]() {
        wg_fft16<T, LOGN, -1, NREG, NT7>(S, twr);
        rows_post_forward<T, LOGN, BC, NREG, NT7>(S, twd);
        wg_fft16_mapped<T, LOGN, -1, NREG, NT7, ColMap<LOGN, BC>>(S, twr);
        cols_symbol_mapped<T, LOGN, BC, NREG, NT7, ColMap<LOGN, BC>>(S, s, eig_l, twd);
        wg_fft16_mapped<T, LOGN, +1, NREG, NT7, ColMap<LOGN, BC>>(S, twr);
        rows_pre_inverse<T, LOGN, BC, NREG, NT7>(S, twd);
        wg_fft16<T, LOGN, +1, NREG, NT7>(S, twr);
    };
    auto Yat = [&](int c, int y, int x) -> T {
        const cplx<T> zv = S[rix<LOGN>(c * H + (y >> 1), pos(x))];
        return (y & 1) ? zv.im : zv.re;
    };

    // ---- primal descent U_{n+1} = U_n - tau_u grad F(U_n)^T P~ with
    // P~ = P_{n+1} + omega (P_{n+1} - P_n), P_{n+1} = P_n + tau_p Y, formed where the
    // stencil reads it, in place on U (the adjoint reads U only at its own point);
    // mixed: on e, with f' at U_b + e.  Then the dual ascent P_{n+1} = P_n + tau_p Y,
    // once every thread has read the P_n it needs.
    auto primal_dual = [&](bool first) {
        const T tu = (T)s.tau_u, tp = (T)s.tau_p, om = (T)s.omega;
        constexpr int CK = wg_chunk<LOGN, C *(SY::NS + 2), (int)sizeof(T)>();
#pragma unroll 1
        for (int i0 = 0; i0 < PPT; i0 += CK) {
            T pt[CK][C][SY::NS], un[CK][C], Uc[CK][C];
#pragma unroll
            for (int j = 0; j < CK; ++j) {
                const int g = pt_of(i0 + j);
                if (g >= NN) continue;
                const int y = g >> LOGN, x = g & (N - 1);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if constexpr (MODE == MODE_F64) {
                        un[j][c] = U[c * NN + g];
                        Uc[j][c] = un[j][c];
                    } else {
                        un[j][c] = first ? (T)0 : U[c * NN + g];
                        Uc[j][c] = (T)Ub[c * NN + g] + un[j][c];
                    }
#pragma unroll
                    for (int q = 0; q < SY::NS; ++q) {
                        const int yy = wrap<BC>(y + SY::dy(q), N), xx = wrap<BC>(x + SY::dx(q), N);
                        const T pn = first ? (T)0 : P[c * NN + yy * N + xx];
                        const T pn1 = pn + tp * Yat(c, yy, xx);
                        pt[j][c][q] = pn1 + om * (pn1 - pn);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < CK; ++j) {
                const int g = pt_of(i0 + j);
                if (g >= NN) continue;
                T adj[C];
                eval_adjoint<EQ, T>(s, [&](int c, int dy, int dx) { return pt[j][c][SY::idx(dy, dx)]; }, Uc[j], adj);
#pragma unroll
                for (int c = 0; c < C; ++c) U[c * NN + g] = un[j][c] - tu * adj[c];
            }
        }
        __syncthreads();
        constexpr int CKP = wg_chunk<LOGN, 2 * C, (int)sizeof(T)>();
#pragma unroll 1
        for (int i0 = 0; i0 < PPT; i0 += CKP) {
            T pn[CKP][C], yv[CKP][C];
#pragma unroll
            for (int j = 0; j < CKP; ++j) {
                const int g = pt_of(i0 + j);
                if (g >= NN) continue;
                const int y = g >> LOGN, x = g & (N - 1);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    pn[j][c] = first ? (T)0 : P[c * NN + g];
                    yv[j][c] = Yat(c, y, x);
                }
            }
#pragma unroll
            for (int j = 0; j < CKP; ++j) {
                const int g = pt_of(i0 + j);
                if (g >= NN) continue;
#pragma unroll
                for (int c = 0; c < C; ++c) P[c * NN + g] = pn[j][c] + tp * yv[j][c];
            }
        }
        __syncthreads();
    };

    // ---- the initial state U_0 = U^k (or the pointwise reaction prox of U^k)
    auto initial = [&](auto *Ui) {
        for (int g = tid; g < NN; g += NT7) {
            if constexpr (EQ == EQ_SCHNAK) {
                double u = src[g], v = src[NN + g];
                if (s.init != 0) prox_schnak(src[g], src[NN + g], s.ht, s.sa, s.sb, s.kappa, u, v);
                Ui[g] = u;
                Ui[NN + g] = v;
            } else {
                Ui[g] = (s.init != 0 && EQ == EQ_LAP5) ? prox_ac(src[g], s.ht, s.b) : src[g];
            }
        }
        __syncthreads();
    };

    if constexpr (MODE == MODE_F64) {
        initial(U);
        residual64(U, [&](double res, double m) { stl = decide<K_INIT64>(stl, rule, res, m); });
        while (!stl.done) {
            const bool first = stl.iters == 0;
            precond();
            primal_dual(first);
            residual64(U, [&](double res, double m) { stl = decide<K_ITER64>(stl, rule, res, m); });
        }
        // the result where the batched path leaves it: U[iters & 1]
        double *out = (double *)s.U[stl.iters & 1];
        if ((void *)out != (void *)U)
            for (int g = tid; g < C * NN; g += NT7) out[g] = U[g];
    } else {
        // outer initial pass: U = U^k (or its prox) in FP64
        initial(U64);
        residual64(U64, [&](double res, double m) { stl = decide<K_OUTER_INIT>(stl, rule, res, m); });
        while (!stl.outer_done) {
            // inner FP32 loop on the correction e (e_0 = 0, P_0 = 0) from W = r
            while (!stl.done) {
                const bool first = stl.iters == 0;
                precond();
                primal_dual(first);
                residual32();
            }
            // outer update U += e, then r = F(U) in FP64 and the outer decision
            if (stl.iters > 0) {
                for (int g = tid; g < C * NN; g += NT7) U64[g] += (double)U[g];
                __syncthreads();
            }
            residual64(U64, [&](double res, double m) { stl = decide<K_OUTER_UPD>(stl, rule, res, m); });
        }
        double *out = s.U64[stl.outer & 1];
        if (out != U64)
            for (int g = tid; g < C * NN; g += NT7) out[g] = U64[g];
    }
    if (tid == 0) store_state(s.st, stl);
}

}  // namespace rdk
