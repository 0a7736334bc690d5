// Workgroup FFT with radix-16 passes, 16 values per thread.
//
// A length-N transform (N = 2^LOGN, 16 <= N <= 4096) is done by N/16 threads
// (one wave or less for N <= 1024, several waves above), in an LDS region of
// N complex values laid out with one padding slot per 16 (index i at
// i + i/16), which keeps the stride-R writes of a Stockham pass off a single
// bank group.  Passes are Stockham autosort passes of radix 16, then one pass
// of radix 8, 4 or 2 for the remaining bits; each thread runs 16/R butterflies
// of a radix-R pass.  The twiddles W^{r k}, r = 1..R-1, of a butterfly are
// products of the gathered powers W^{k}, W^{2k}, W^{4k}, W^{8k}, so a
// butterfly gathers at most 4 table entries and each twiddle carries at most
// 3 roundings.
#pragma once
#include "fft.h"

namespace rdk {

template <typename T, int DIR> __device__ __forceinline__ void dft16(cplx<T> *v) {
    // radix-4 x radix-4: columns of 4 (stride 4), twiddle W16^{n1 k2}, rows of 4
    cplx<T> a[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) a[n1][n2] = v[n1 + 4 * n2];
        dft4<T, DIR>(a[n1]);   // over n2 -> k2
    }
    const T c1 = (T)0.923879532511286756128183189396788934;   // cos(pi/8)
    const T s1 = (T)0.382683432365089771728459984030398867;   // sin(pi/8)
    const T r2 = (T)0.707106781186547524400844362104849039;
    const T d = (T)DIR;
    // W16^{m} = cos(2 pi m/16) + DIR i sin(2 pi m/16), for m = n1 * k2
    auto tw16 = [&](int m) -> cplx<T> {
        switch (m) {
        case 1: return {c1, d * s1};
        case 2: return {r2, d * r2};
        case 3: return {s1, d * c1};
        case 4: return {(T)0, d};
        case 6: return {-r2, d * r2};
        case 9: return {-c1, -d * s1};
        default: return {(T)1, (T)0};
        }
    };
#pragma unroll
    for (int n1 = 1; n1 < 4; ++n1)
#pragma unroll
        for (int k2 = 1; k2 < 4; ++k2) a[n1][k2] = cmul(a[n1][k2], tw16(n1 * k2));
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        cplx<T> b[4] = {a[0][k2], a[1][k2], a[2][k2], a[3][k2]};
        dft4<T, DIR>(b);   // over n1 -> k1
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) v[k2 + 4 * k1] = b[k1];
    }
}

template <typename T, int R, int DIR> __device__ __forceinline__ void dftR(cplx<T> *v) {
    if constexpr (R == 16) dft16<T, DIR>(v);
    else if constexpr (R == 8) dft8<T, DIR>(v);
    else if constexpr (R == 4) dft4<T, DIR>(v);
    else dft2<T, DIR>(v);
}

// Radix and butterfly count of pass q of a length-2^LOGN transform: radix 16
// while at least 4 bits remain, then one pass of radix 8, 4 or 2.
template <int LOGN> constexpr int npasses16() { return (LOGN + 3) / 4; }
template <int LOGN> constexpr int pass_radix(int q) { return LOGN - 4 * q >= 4 ? 16 : (1 << (LOGN - 4 * q)); }

// The twiddles of one thread for every pass after the first: for butterfly b of
// pass q, the gathered powers W^{k}, W^{2k}, W^{4k}, W^{8k} (forward sign) of
// W = exp(-2 pi i / (NS R)), k = j mod NS.  They depend only on the thread's
// index in its transform team, so a kernel loads them once, at its start, and
// every transform (forward and inverse) of the kernel reuses them.
template <typename T, int LOGN> struct Tw16 {
    cplx<T> p[npasses16<LOGN>() > 1 ? npasses16<LOGN>() - 1 : 1][8][4];
};

template <typename T, int LOGN>
__device__ __forceinline__ void load_tw16(Tw16<T, LOGN> &w, const cplx<T> *__restrict__ tw, int t) {
    constexpr int N = 1 << LOGN;
    constexpr int TPF = N / 16;
    const auto tg = gp(tw);
#pragma unroll
    for (int q = 1; q < npasses16<LOGN>(); ++q) {
        const int R = pass_radix<LOGN>(q), NS = 1 << (4 * q);
        const int TWSTEP = N / (NS * R);
#pragma unroll
        for (int b = 0; b < 16 / R; ++b) {
            const int k = (t + b * TPF) & (NS - 1);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if ((1 << e) < R) {
                    const int i = ((k * TWSTEP) << e) & (N - 1);
                    w.p[q - 1][b][e] = {tg[i].re, tg[i].im};
                }
        }
    }
}

template <typename T, int LOGN>
__device__ __forceinline__ void load_tw16(Tw16<T, LOGN> &w, const cplx<T> *__restrict__ tw) {
    load_tw16<T, LOGN>(w, tw, (int)(threadIdx.x % ((1 << LOGN) / 16)));
}

// One Stockham pass of radix R (NS = product of earlier radices).  Butterfly j
// reads x[j + r N/R], twiddles input r by W_{NS R}^{r k} (k = j mod NS), applies
// DFT_R, and writes output q to ((j - k) R + k) + q NS.  pw: the thread's
// gathered powers for this pass (unused when NS = 1).  Thread t of a transform
// runs butterflies j = t + b N/16, b < 16/R.
//
// pass_in: the reads, twiddles and butterflies of the thread (outputs in v).
template <typename T, int LOGN, int R, int NS, int DIR>
__device__ __forceinline__ void pass_in(const cplx<T> *x, int t, const cplx<T> (*pw)[4], cplx<T> (*v)[R]) {
    constexpr int N = 1 << LOGN;
    constexpr int TPF = N / 16;      // threads per transform
    constexpr int NB = N / R;        // butterflies
    constexpr int BPT = 16 / R;      // butterflies per thread
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int j = t + b * TPF;
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = x[lds_pad(j + r * NB)];
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

// pass_out: the Stockham writes of the thread's butterfly outputs.
template <typename T, int LOGN, int R, int NS>
__device__ __forceinline__ void pass_out(cplx<T> *x, int t, const cplx<T> (*v)[R]) {
    constexpr int TPF = (1 << LOGN) / 16;
#pragma unroll
    for (int b = 0; b < 16 / R; ++b) {
        const int j = t + b * TPF;
        const int k = j & (NS - 1);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) x[lds_pad(base + q * NS)] = v[b][q];
    }
}

template <typename T, int LOGN, int R, int NS, int DIR>
__device__ __forceinline__ void pass16(cplx<T> *x, int t, bool active, const cplx<T> (*pw)[4]) {
    cplx<T> v[16 / R][R];
    if (active) pass_in<T, LOGN, R, NS, DIR>(x, t, pw, v);
    __syncthreads();
    if (active) pass_out<T, LOGN, R, NS>(x, t, v);
    __syncthreads();
}

template <typename T, int LOGN, int DIR, int DONE>
__device__ __forceinline__ void passes16(cplx<T> *x, int t, bool active, const Tw16<T, LOGN> &w) {
    if constexpr (DONE < LOGN) {
        constexpr int REM = LOGN - DONE;
        constexpr int R = REM >= 4 ? 16 : (1 << REM);
        constexpr int LOGR = REM >= 4 ? 4 : REM;
        constexpr int q = DONE / 4;
        pass16<T, LOGN, R, (1 << DONE), DIR>(x, t, active, w.p[q > 0 ? q - 1 : 0]);
        passes16<T, LOGN, DIR, DONE + LOGR>(x, t, active, w);
    }
}

// ---- transforms whose first input and last output stay in registers
//
// Thread t of a transform holds its 16 values in "stride order": value r is
// element t + r N/16.  That is what the first radix-16 pass reads (NS = 1,
// butterfly j = t) and, for the last pass of radix RL (NS = N/RL, butterflies
// j = t + b N/16 with k = j), output q of butterfly b lands at
// t + (b + q 16/RL) N/16, again element t + r N/16 with r = b + q 16/RL.  So a
// transform can start from values loaded straight from global memory and end
// with values ready to be stored, with LDS used only between passes.

// Radix of the last pass and the register index of its output (b, q).
template <int LOGN> constexpr int last_radix() { return pass_radix<LOGN>(npasses16<LOGN>() - 1); }
template <int LOGN> __host__ __device__ constexpr int last_slot(int b, int q) { return b + q * (16 / last_radix<LOGN>()); }

// Middle passes q = 1 .. npasses - 2 (all radix 16), each ending with a barrier.
template <typename T, int LOGN, int DIR, int Q>
__device__ __forceinline__ void middle_passes(cplx<T> *x, int t, const Tw16<T, LOGN> &w) {
    if constexpr (Q < npasses16<LOGN>() - 1) {
        pass16<T, LOGN, 16, (1 << (4 * Q)), DIR>(x, t, true, w.p[Q - 1]);
        middle_passes<T, LOGN, DIR, Q + 1>(x, t, w);
    }
}

// Transform of one region x whose input v (stride order) is in registers; the
// output is left in v (stride order).  Needs at least two passes.  Starts by
// writing x (the caller makes sure no thread still reads it) and ends with the
// last pass's reads of x (the caller places a barrier before x is rewritten).
template <typename T, int LOGN, int DIR>
__device__ __forceinline__ void fft16_regs(cplx<T> *x, int t, const Tw16<T, LOGN> &w, cplx<T> *v) {
    static_assert(npasses16<LOGN>() >= 2, "register-ended transforms need two passes");
    constexpr int NP = npasses16<LOGN>();
    constexpr int RL = last_radix<LOGN>();
    dft16<T, DIR>(v);
#pragma unroll
    for (int q = 0; q < 16; ++q) x[lds_pad(16 * t + q)] = v[q];
    __syncthreads();
    middle_passes<T, LOGN, DIR, 1>(x, t, w);
    cplx<T> o[16 / RL][RL];
    pass_in<T, LOGN, RL, (1 << (4 * (NP - 1))), DIR>(x, t, w.p[NP - 2], o);
#pragma unroll
    for (int b = 0; b < 16 / RL; ++b)
#pragma unroll
        for (int q = 0; q < RL; ++q) v[last_slot<LOGN>(b, q)] = o[b][q];
}

// In-place transforms of NREG regions (region i at buf + i * lds_region<LOGN>(),
// padded indexing) by a workgroup of NTH threads; teams of N/16 threads take
// regions round-robin.  Ends with a barrier.  DIR -1 forward, +1 inverse.
// w: the thread's twiddles (load_tw16).
template <typename T, int LOGN, int DIR, int NREG, int NTH>
__device__ __forceinline__ void wg_fft16(cplx<T> *buf, const Tw16<T, LOGN> &w) {
    constexpr int TPF = (1 << LOGN) / 16;
    static_assert(NTH % TPF == 0 || TPF > NTH, "team must divide the workgroup");
    constexpr int NTEAMS = NTH / TPF;
    const int team = threadIdx.x / TPF, t = threadIdx.x % TPF;
#pragma unroll 1
    for (int g = 0; g < NREG; g += NTEAMS) {
        const int reg = g + team;
        const bool active = reg < NREG;
        passes16<T, LOGN, DIR, 0>(buf + (active ? reg : 0) * lds_region<LOGN>(), t, active, w);
    }
}

}  // namespace rdk
