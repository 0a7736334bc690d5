// Small grids: one workgroup runs a whole implicit step.
//
// On N <= 128 grids an iteration moves a few hundred KB, and the four launches of
// the batched iteration (column pass, inverse rows, primal update, forward rows)
// cost their launch latency, not their bytes.  Here one workgroup per slot takes
// the whole step, Algorithm 1 with its stop test, in one launch:
//
//   W = F(U_n) (stencil)  -> spectrum S in LDS (row pairs packed as complex rows)
//   ||W / h_t|| (fixed-order workgroup sum), stop decision (decide<>, thread 0)
//   row FFTs, column FFTs (on the row layout), 1 / (N^2 g), inverse column
//   FFTs, inverse row FFTs                          -> Y = G^-1 W_n in LDS
//   P_{n+1} = P_n + tau_p Y,  P~ = P_{n+1} + omega tau_p Y (P~ kept in LDS)
//   U_{n+1} = U_n - tau_u grad F(U_n)^T P~
//
// and, in the mixed precision, the same FP32 inner loop on the correction e with
// the FP64 outer passes (U += e, r = F(U), stop test) between inner loops.  The
// spectrum always lives in LDS; the iterate, P and (mixed) the FP32 copies of U
// and r take LDS in that order while the 160 KB of a gfx950 workgroup allow, and
// otherwise stay in the slot's HBM buffers (then L2-resident).  The arithmetic
// per point is that of the batched kernels (the same eval_F / eval_Ftilde /
// eval_adjoint code, the pair / cosine processing and symbol of fft.h); the
// transforms are radix-8 passes and the norm's sums run in another order.
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
// region c H + y / 2.  The transforms below take an address map, so no transpose
// is needed between the row and the column transforms.
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

// ---------------------------------------------------------------- radix-8 transforms
// The single-workgroup step's transforms (N <= 64): Stockham passes of radix 8 while
// three bits remain, then one of radix 4 or 2, with 8 values per thread (N/8 threads
// per transform: twice the threads of the radix-16 passes on these short
// transforms, whose passes are bound by arithmetic latency, not LDS).  Pass q reads
// element j + r N/R of butterfly j, multiplies input r by W_{NS R}^{r k} (k = j mod
// NS), applies DFT_R and writes output q to (j - k) R + k + q NS.  The twiddles of a
// thread depend only on its index in its team, so they are read from the table
// exp(-2 pi i m / N) once per step and kept in registers; the inverse conjugates.
template <int LOGN> constexpr int r8_radix(int q) { return LOGN - 3 * q >= 3 ? 8 : (1 << (LOGN - 3 * q)); }
template <int LOGN> constexpr int r8_passes() { return (LOGN + 2) / 3; }

template <typename T, int LOGN> struct TwR8 {
    // pass 1 (the only pass with NS > 1 for N <= 64): butterflies b < 8 / R, inputs 1..R-1
    cplx<T> w[4][7];
};

template <typename T, int LOGN>
__device__ __forceinline__ void load_twr8(TwR8<T, LOGN> &tw, const cplx<T> *table) {
    static_assert(r8_passes<LOGN>() <= 2, "radix-8 step transforms: N <= 64");
    constexpr int N = 1 << LOGN, TPT = N / 8;
    if constexpr (r8_passes<LOGN>() == 2) {
        constexpr int R = r8_radix<LOGN>(1), NS = 8, NB = N / R, BPT = 8 / R;
        constexpr int STEP = N / (NS * R);
        const int t = threadIdx.x % TPT;
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int j = t + b * TPT;
            const int k = j & (NS - 1);
            (void)NB;
#pragma unroll
            for (int r = 1; r < R; ++r) tw.w[b][r - 1] = table[(r * k * STEP) & (N - 1)];
        }
    }
}

template <typename T, int LOGN, int Q, int DIR, class M>
__device__ __forceinline__ void r8_pass(cplx<T> *buf, int reg, int t, bool active, const TwR8<T, LOGN> &tw) {
    constexpr int N = 1 << LOGN, TPT = N / 8;
    constexpr int R = r8_radix<LOGN>(Q), NS = Q == 0 ? 1 : 8, NB = N / R, BPT = 8 / R;
    cplx<T> v[BPT][R];
    if (active) {
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int j = t + b * TPT;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = buf[M::at(reg, j + r * NB)];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const cplx<T> w = DIR < 0 ? tw.w[b][r - 1] : cconj(tw.w[b][r - 1]);
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
            const int j = t + b * TPT;
            const int k = j & (NS - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[M::at(reg, base + q * NS)] = v[b][q];
        }
    }
    __syncthreads();
}

// In-place transforms of NREG regions (address map M) by NTH threads; teams of N/8
// threads take regions round-robin.  Ends with a barrier.
template <typename T, int LOGN, int DIR, int NREG, int NTH, class M>
__device__ __forceinline__ void wg_fft_r8(cplx<T> *buf, const TwR8<T, LOGN> &tw) {
    constexpr int TPT = (1 << LOGN) / 8;
    constexpr int NTEAMS = NTH / TPT;
    const int team = threadIdx.x / TPT, t = threadIdx.x % TPT;
#pragma unroll 1
    for (int g = 0; g < NREG; g += NTEAMS) {
        const int reg = g + team;
        const bool active = reg < NREG;
        r8_pass<T, LOGN, 0, DIR, M>(buf, active ? reg : 0, t, active, tw);
        if constexpr (r8_passes<LOGN>() == 2) r8_pass<T, LOGN, 1, DIR, M>(buf, active ? reg : 0, t, active, tw);
    }
}

template <int LOGN> struct RowMap {
    __device__ __forceinline__ static int at(int reg, int i) { return rix<LOGN>(reg, i); }
};

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

// Strips: in the point phases thread t takes rows y0 .. y0 + L - 1 of column
// x = t mod N (L = N^2 / NT7, at least 1), in sub-strips of LS rows whose stencil
// neighbourhood (reach HY, the diamond |dy| + |dx| <= HY: 5 or 13 points) it loads
// into registers once.  The rows of a sub-strip pair up (2q, 2q + 1), the two rows
// a complex slot of the spectrum packs, so W and Y move as one complex value.
template <int LOGN> constexpr int wg_strip() { return (1 << (2 * LOGN)) >= NT7 ? (1 << (2 * LOGN)) / NT7 : 1; }
template <int LOGN, int HY, int C> constexpr int wg_substrip() {
    constexpr int L = wg_strip<LOGN>();
    constexpr int cap = (HY >= 2 || C == 2) ? 2 : 8;   // windows within the register budget
    return L < cap ? L : cap;
}
// Whether window row r (-HY .. LS - 1 + HY) at column offset dx is in the
// neighbourhood of some row of a sub-strip of LS rows.
template <int HY, int LS> __host__ __device__ constexpr bool wg_needed(int r, int dx) {
    const int dist = r < 0 ? -r : (r >= LS ? r - LS + 1 : 0);
    return dist + (dx < 0 ? -dx : dx) <= HY;
}

template <typename T, int LOGN, int BC, int EQ, int MODE>
__global__ __launch_bounds__(NT7) void k_step_wg(Slot *const *slots) {
    constexpr int C = EQ == EQ_SCHNAK ? 2 : 1;
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int NN = N * N;
    constexpr int NREG = C * H;   // row-pair regions = column regions
    constexpr int HY = stencil_hy<EQ>();
    constexpr int HU = EQ == EQ_BIH ? 1 : 0;   // reach of U in the mixed inner residual
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
    TwR8<T, LOGN> twr;
    load_twr8<T, LOGN>(twr, (const cplx<T> *)s.tw);
    const StopRule rule{s.tol, s.inner_rtol, s.max_iter, s.max_outer};
    auto pos = [](int x) { return BC == BC_P ? x : dct_pos(x, N); };
    auto at = [](int c, int y, int x) { return c * NN + wrap<BC>(y, N) * N + wrap<BC>(x, N); };
    constexpr int L = wg_strip<LOGN>();
    constexpr int LS = wg_substrip<LOGN, HY, C>();
    constexpr int STRIP_THREADS = N * (N / L);
    static_assert(L % LS == 0 && (LS == 1 || LS % 2 == 0), "sub-strips of whole row pairs");
    // W of rows ys .. ys + LS - 1 at column x into the spectrum's row-pair layout
    auto store_w = [&](int c, int ys, int x, const double *W) {
        if constexpr (LS >= 2) {
#pragma unroll
            for (int q = 0; q < LS / 2; ++q)
                S[rix<LOGN>(c * H + (ys >> 1) + q, pos(x))] = cplx<T>{(T)W[2 * q], (T)W[2 * q + 1]};
        } else {
            rreal<T, LOGN>(S, c * H + ys / 2, 2 * pos(x) + (ys & 1)) = (T)W[0];
        }
    };
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
        double acc[2 * C];
#pragma unroll
        for (int k = 0; k < 2 * C; ++k) acc[k] = 0.0;
        if (tid < STRIP_THREADS) {
            const int x = tid % N, y0 = (tid / N) * L;
#pragma unroll 1
            for (int s0 = 0; s0 < L; s0 += LS) {
                const int ys = y0 + s0;
                double v[C][LS + 2 * HY][2 * HY + 1], uk[C][LS];
#pragma unroll
                for (int c = 0; c < C; ++c) {
#pragma unroll
                    for (int r = -HY; r < LS + HY; ++r)
#pragma unroll
                        for (int dx = -HY; dx <= HY; ++dx)
                            if (wg_needed<HY, LS>(r, dx)) v[c][r + HY][dx + HY] = Uf[at(c, ys + r, x + dx)];
#pragma unroll
                    for (int i = 0; i < LS; ++i) uk[c][i] = Ukp[c * NN + (ys + i) * N + x];
                }
                double W[C][LS];
#pragma unroll
                for (int i = 0; i < LS; ++i) {
                    double Wi[C], Uc[C], ukc[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) ukc[c] = uk[c][i];
                    eval_F<EQ, double>(s, [&](int c, int dy, int dx) { return v[c][i + dy + HY][dx + HY]; }, ukc, Wi,
                                       Uc);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        W[c][i] = Wi[c];
                        acc[c] += Wi[c] * Wi[c];
                        acc[C + c] += Uc[c] - ukc[c];
                        if constexpr (MODE == MODE_MIXED) {
                            Rr[c * NN + (ys + i) * N + x] = (float)Wi[c];
                            Ub[c * NN + (ys + i) * N + x] = (float)Uc[c];
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < C; ++c) store_w(c, ys, x, W[c]);
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
        double acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0.0;
        if (tid < STRIP_THREADS) {
            const int x = tid % N, y0 = (tid / N) * L;
#pragma unroll 1
            for (int s0 = 0; s0 < L; s0 += LS) {
                const int ys = y0 + s0;
                float ve[C][LS + 2 * HY][2 * HY + 1], vu[C][LS + 2 * HU][2 * HU + 1], rc[C][LS];
#pragma unroll
                for (int c = 0; c < C; ++c) {
#pragma unroll
                    for (int r = -HY; r < LS + HY; ++r)
#pragma unroll
                        for (int dx = -HY; dx <= HY; ++dx)
                            if (wg_needed<HY, LS>(r, dx)) ve[c][r + HY][dx + HY] = (float)U[at(c, ys + r, x + dx)];
#pragma unroll
                    for (int r = -HU; r < LS + HU; ++r)
#pragma unroll
                        for (int dx = -HU; dx <= HU; ++dx)
                            if (wg_needed<HU, LS>(r, dx)) vu[c][r + HU][dx + HU] = Ub[at(c, ys + r, x + dx)];
#pragma unroll
                    for (int i = 0; i < LS; ++i) rc[c][i] = Rr[c * NN + (ys + i) * N + x];
                }
                double W[C][LS];
#pragma unroll
                for (int i = 0; i < LS; ++i) {
                    float Wi[C], r[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) r[c] = rc[c][i];
                    eval_Ftilde<EQ>(s, [&](int c, int dy, int dx) { return ve[c][i + dy + HY][dx + HY]; },
                                    [&](int c, int dy, int dx) { return vu[c][i + dy + HU][dx + HU]; }, r, Wi);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        W[c][i] = Wi[c];
                        acc[c] += (double)Wi[c] * (double)Wi[c];
                    }
                }
#pragma unroll
                for (int c = 0; c < C; ++c) store_w(c, ys, x, W[c]);
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
        wg_fft_r8<T, LOGN, -1, NREG, NT7, RowMap<LOGN>>(S, twr);
        rows_post_forward<T, LOGN, BC, NREG, NT7>(S, twd);
        wg_fft_r8<T, LOGN, -1, NREG, NT7, ColMap<LOGN, BC>>(S, twr);
        cols_symbol_mapped<T, LOGN, BC, NREG, NT7, ColMap<LOGN, BC>>(S, s, eig_l, twd);
        wg_fft_r8<T, LOGN, +1, NREG, NT7, ColMap<LOGN, BC>>(S, twr);
        rows_pre_inverse<T, LOGN, BC, NREG, NT7>(S, twd);
        wg_fft_r8<T, LOGN, +1, NREG, NT7, RowMap<LOGN>>(S, twr);
    };
    auto Yat = [&](int c, int y, int x) -> T {
        const cplx<T> zv = S[rix<LOGN>(c * H + (y >> 1), pos(x))];
        return (y & 1) ? zv.im : zv.re;
    };

    // ---- primal descent U_{n+1} = U_n - tau_u grad F(U_n)^T P~ with
    // P~ = P_{n+1} + omega (P_{n+1} - P_n), P_{n+1} = P_n + tau_p Y, formed in the
    // registers of the strip that reads it, in place on U (the adjoint reads U only
    // at its own point); mixed: on e, with f' at U_b + e.  Then the dual ascent:
    // P_{n+1} of the strip's own points, stored once every thread has read the P_n
    // it needs.
    auto primal_dual = [&](bool first) {
        const T tu = (T)s.tau_u, tp = (T)s.tau_p, om = (T)s.omega;
        T pnew[C][L];
        if (tid < STRIP_THREADS) {
            const int x = tid % N, y0 = (tid / N) * L;
#pragma unroll
            for (int s0 = 0; s0 < L; s0 += LS) {
                const int ys = y0 + s0;
                T pt[C][LS + 2 * HY][2 * HY + 1];
                auto cell = [&](int c, int r, int dx, int yy, int xx, T Y) {
                    const T pn = first ? (T)0 : P[c * NN + yy * N + xx];
                    const T pn1 = pn + tp * Y;
                    pt[c][r + HY][dx + HY] = pn1 + om * (pn1 - pn);
                    if (dx == 0 && r >= 0 && r < LS) pnew[c][s0 + r] = pn1;
                };
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int dx = -HY; dx <= HY; ++dx) {
                        const int xx = wrap<BC>(x + dx, N), px = pos(xx);
                        if constexpr (LS >= 2) {
                            // the strip's own rows, two per complex slot
#pragma unroll
                            for (int q = 0; q < LS / 2; ++q) {
                                const cplx<T> z = S[rix<LOGN>(c * H + (ys >> 1) + q, px)];
                                cell(c, 2 * q, dx, ys + 2 * q, xx, z.re);
                                cell(c, 2 * q + 1, dx, ys + 2 * q + 1, xx, z.im);
                            }
                        } else {
                            const cplx<T> z = S[rix<LOGN>(c * H + (ys >> 1), px)];
                            cell(c, 0, dx, ys, xx, (ys & 1) ? z.im : z.re);
                        }
                        // halo rows, through the boundary map
#pragma unroll
                        for (int r = -HY; r < LS + HY; ++r) {
                            if (r >= 0 && r < LS) continue;
                            if (!wg_needed<HY, LS>(r, dx)) continue;
                            const int yy = wrap<BC>(ys + r, N);
                            const cplx<T> z = S[rix<LOGN>(c * H + (yy >> 1), px)];
                            cell(c, r, dx, yy, xx, (yy & 1) ? z.im : z.re);
                        }
                    }
#pragma unroll
                for (int i = 0; i < LS; ++i) {
                    const int g = (ys + i) * N + x;
                    T un[C], Uc[C], adj[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        if constexpr (MODE == MODE_F64) {
                            un[c] = U[c * NN + g];
                            Uc[c] = un[c];
                        } else {
                            un[c] = first ? (T)0 : U[c * NN + g];
                            Uc[c] = (T)Ub[c * NN + g] + un[c];
                        }
                    }
                    eval_adjoint<EQ, T>(s, [&](int c, int dy, int dx) { return pt[c][i + dy + HY][dx + HY]; }, Uc,
                                        adj);
#pragma unroll
                    for (int c = 0; c < C; ++c) U[c * NN + g] = un[c] - tu * adj[c];
                }
            }
        }
        __syncthreads();
        if (tid < STRIP_THREADS) {
            const int x = tid % N, y0 = (tid / N) * L;
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int i = 0; i < L; ++i) P[c * NN + (y0 + i) * N + x] = pnew[c][i];
        }
        // the next reader of P is the next primal step, several barriers later
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
