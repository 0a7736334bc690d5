// Workgroup FFTs in LDS and the real-data / cosine-transform wrappers around them.
//
// The preconditioner G is diagonal in the 2-D DFT basis (periodic grids) and in
// the 2-D DCT-II basis (Neumann grids) (Sec. 2.1, "Application of FFT"; Remark 1).
// Both are computed here from complex FFTs of length N:
//
//  * Two real rows a, b are packed as one complex row z = a + i b.  From
//    Z = FFT(z) the two half spectra are A_k = (Z_k + conj Z_{N-k}) / 2 and
//    B_k = (Z_k - conj Z_{N-k}) / (2i).  A row's N/2 + 1 bins are stored as N/2
//    complex slots, slot 0 holding the two real bins (A_0, A_{N/2}).
//  * DCT-II (unnormalised, X_k = sum_n x_n cos(pi k (2n+1) / (2N))) by Makhoul's
//    method: reorder v_n = x_{2n}, v_{N-1-n} = x_{2n+1}, V = FFT(v), then
//    X_k = Re(w_k V_k) and X_{N-k} = -Im(w_k V_k) with w_k = exp(-i pi k / (2N)).
//    The inverse rebuilds V_k = conj(w_k) (X_k - i X_{N-k}) (X_N = 0) and applies
//    an inverse FFT.  Two real sequences are again packed into one complex FFT.
//
// FFTs are Stockham autosort passes (radix 8, then one radix-4 or radix-2 pass),
// forward sign -1, both directions unnormalised; the 1/N^2 of the 2-D inverse is
// folded into the symbol multiplier.
#pragma once
#include "rd_dev.h"

namespace rdk {

template <typename T, int DIR> __device__ __forceinline__ cplx<T> rot90(cplx<T> a) {
    // multiply by exp(DIR i pi / 2): -i for the forward transform, +i for the inverse
    return DIR < 0 ? cplx<T>{a.im, -a.re} : cplx<T>{-a.im, a.re};
}

template <typename T, int DIR> __device__ __forceinline__ void dft2(cplx<T> *v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, int DIR> __device__ __forceinline__ void dft4(cplx<T> *v) {
    cplx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    cplx<T> t2 = cadd(v[1], v[3]), t3 = rot90<T, DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <typename T, int DIR> __device__ __forceinline__ void dft8(cplx<T> *v) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<T, DIR>(e);
    dft4<T, DIR>(o);
    const T s = (T)0.707106781186547524400844362104849039;
    const T d = (T)DIR;
    // o_q * exp(DIR i pi q / 4) for q = 1, 2, 3
    cplx<T> o1 = {s * (o[1].re - d * o[1].im), s * (o[1].im + d * o[1].re)};
    cplx<T> o2 = rot90<T, DIR>(o[2]);
    cplx<T> o3 = {s * (-o[3].re - d * o[3].im), s * (-o[3].im + d * o[3].re)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <typename T, int R, int DIR> __device__ __forceinline__ void dft(cplx<T> *v) {
    if constexpr (R == 8) dft8<T, DIR>(v);
    else if constexpr (R == 4) dft4<T, DIR>(v);
    else dft2<T, DIR>(v);
}

// One Stockham pass of radix R over a length-N region (NS = product of the
// radices of the passes already done).  Butterfly j reads x[j + r N/R], twiddles
// input r by W_{NS R}^{r k} (k = j mod NS), applies DFT_R and writes output q to
// ((j - k) R + k) + q NS.  Reads complete (barrier) before any write.
template <typename T, int LOGN, int R, int NS, int DIR>
__device__ __forceinline__ void stockham_pass(cplx<T> *x, int lane, bool active,
                                              const cplx<T> *__restrict__ tw) {
    constexpr int N = 1 << LOGN;
    constexpr int TEAM = fft_team<LOGN>();
    constexpr int NB = N / R;
    constexpr int BPT = NB / TEAM;
    constexpr int TWSTEP = N / (NS * R);
    static_assert(BPT >= 1, "team larger than butterfly count");
    cplx<T> v[BPT][R];
    if (active) {
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int j = lane + b * TEAM;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = x[j + r * NB];
            if constexpr (NS > 1) {
                const int k = j & (NS - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cplx<T> w = tw[r * k * TWSTEP];
                    if constexpr (DIR > 0) w.im = -w.im;
                    v[b][r] = cmul(v[b][r], w);
                }
            }
            dft<T, R, DIR>(v[b]);
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int j = lane + b * TEAM;
            const int k = j & (NS - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) x[base + q * NS] = v[b][q];
        }
    }
    __syncthreads();
}

template <typename T, int LOGN, int DIR, int DONE>
__device__ __forceinline__ void stockham_all(cplx<T> *x, int lane, bool active, const cplx<T> *tw) {
    if constexpr (DONE < LOGN) {
        constexpr int REM = LOGN - DONE;
        constexpr int R = REM >= 3 ? 8 : (REM == 2 ? 4 : 2);
        constexpr int LOGR = R == 8 ? 3 : (R == 4 ? 2 : 1);
        stockham_pass<T, LOGN, R, (1 << DONE), DIR>(x, lane, active, tw);
        stockham_all<T, LOGN, DIR, DONE + LOGR>(x, lane, active, tw);
    }
}

// In-place length-N FFTs of NREG regions (region i at buf + i * N) by the whole
// workgroup; teams of fft_team<LOGN>() threads take regions round-robin.
// Ends with a barrier.  DIR = -1 forward, +1 inverse (unnormalised).
template <typename T, int LOGN, int DIR, int NREG>
__device__ __forceinline__ void wg_fft(cplx<T> *buf, const cplx<T> *__restrict__ tw) {
    constexpr int N = 1 << LOGN;
    constexpr int TEAM = fft_team<LOGN>();
    constexpr int NTEAMS = NT / TEAM;
    const int team = threadIdx.x / TEAM;
    const int lane = threadIdx.x % TEAM;
#pragma unroll 1
    for (int g = 0; g < NREG; g += NTEAMS) {
        const int reg = g + team;
        const bool active = reg < NREG;
        stockham_all<T, LOGN, DIR, 0>(buf + (active ? reg : 0) * N, lane, active, tw);
    }
}

// Work items for the pair steps: item (region, l), l < N/2, owns bins l and N-l
// (item 0 owns bins 0 and N/2).
template <int LOGN, int NREG> constexpr int pair_items_per_thread() {
    constexpr int total = NREG * ((1 << LOGN) / 2);
    return (total + NT - 1) / NT;
}

// ---- row pass, forward: packed pair spectrum Z -> two rows of slots (in place).
// Periodic: slots of row a hold (A_0, A_{N/2}) then A_1..A_{N/2-1}; row b likewise.
// Neumann: the region, viewed as 2N reals, holds X_a[0..N) then X_b[0..N).
template <typename T, int LOGN, int BC, int NREG>
__device__ __forceinline__ void rows_post_forward(cplx<T> *buf, const cplx<T> *__restrict__ twd) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int IPT = pair_items_per_thread<LOGN, NREG>();
    cplx<T> oa[IPT], ob[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NT;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        const cplx<T> *z = buf + reg * N;
        if (l == 0) {
            const cplx<T> z0 = z[0], zh = z[H];
            if constexpr (BC == BC_P) {
                oa[i] = {z0.re, zh.re};
                ob[i] = {z0.im, zh.im};
            } else {
                const T s = (T)0.707106781186547524400844362104849039;
                oa[i] = {z0.re, s * zh.re};   // X_a[0], X_a[N/2]
                ob[i] = {z0.im, s * zh.im};
            }
        } else {
            const cplx<T> zl = z[l], zn = z[N - l];
            const cplx<T> A = {(zl.re + zn.re) * (T)0.5, (zl.im - zn.im) * (T)0.5};
            const cplx<T> B = {(zl.im + zn.im) * (T)0.5, (zn.re - zl.re) * (T)0.5};
            if constexpr (BC == BC_P) {
                oa[i] = A;
                ob[i] = B;
            } else {
                const cplx<T> w = twd[l];
                const cplx<T> qa = cmul(A, w), qb = cmul(B, w);
                oa[i] = {qa.re, -qa.im};      // X_a[l], X_a[N-l]
                ob[i] = {qb.re, -qb.im};
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NT;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        cplx<T> *z = buf + reg * N;
        if constexpr (BC == BC_P) {
            z[l] = oa[i];
            z[H + l] = ob[i];
        } else {
            T *xa = reinterpret_cast<T *>(z);
            T *xb = xa + N;
            if (l == 0) {
                xa[0] = oa[i].re; xa[H] = oa[i].im;
                xb[0] = ob[i].re; xb[H] = ob[i].im;
            } else {
                xa[l] = oa[i].re; xa[N - l] = oa[i].im;
                xb[l] = ob[i].re; xb[N - l] = ob[i].im;
            }
        }
    }
    __syncthreads();
}

// ---- row pass, inverse: two rows of slots -> packed pair spectrum Z (in place).
template <typename T, int LOGN, int BC, int NREG>
__device__ __forceinline__ void rows_pre_inverse(cplx<T> *buf, const cplx<T> *__restrict__ twd) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int IPT = pair_items_per_thread<LOGN, NREG>();
    cplx<T> zl_out[IPT], zn_out[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NT;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        const cplx<T> *z = buf + reg * N;
        if constexpr (BC == BC_P) {
            const cplx<T> a = z[l], b = z[H + l];
            if (l == 0) {
                zl_out[i] = {a.re, b.re};   // Z_0 = A_0 + i B_0
                zn_out[i] = {a.im, b.im};   // Z_{N/2}
            } else {
                zl_out[i] = {a.re - b.im, a.im + b.re};
                zn_out[i] = {a.re + b.im, b.re - a.im};
            }
        } else {
            const T *xa = reinterpret_cast<const T *>(z);
            const T *xb = xa + N;
            if (l == 0) {
                const T r2 = (T)1.41421356237309504880168872420969808;
                zl_out[i] = {xa[0], xb[0]};
                zn_out[i] = {r2 * xa[H], r2 * xb[H]};
            } else {
                const cplx<T> wc = cconj(twd[l]);
                const cplx<T> va = cmul(wc, cplx<T>{xa[l], -xa[N - l]});
                const cplx<T> vb = cmul(wc, cplx<T>{xb[l], -xb[N - l]});
                zl_out[i] = {va.re - vb.im, va.im + vb.re};
                zn_out[i] = {va.re + vb.im, vb.re - va.im};
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NT;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        cplx<T> *z = buf + reg * N;
        z[l] = zl_out[i];
        z[l == 0 ? H : N - l] = zn_out[i];
    }
    __syncthreads();
}

// Symbol multiplier 1 / (N^2 g), g = (1 + alpha mu + beta mu^2)^2, mu = s_kx + s_ky.
__device__ __forceinline__ double symbol_mult(const double *__restrict__ eig, int kx, int ky, double alpha,
                                              double beta, double invN2) {
    const double mu = eig[kx] + eig[ky];
    const double a = 1.0 + alpha * mu + beta * mu * mu;
    return invN2 / (a * a);
}

// ---- column pass, between the forward and inverse column FFTs: multiply by the
// symbol.  Region `reg` holds column job (component c, column j) with
// c = job / H, j = job % H.  Periodic: column j is the row spectrum at kx = j;
// column 0 packs kx = 0 (real part) and kx = N/2 (imaginary part).  Neumann:
// column j packs kx = 2j (real) and kx = 2j + 1 (imaginary), both cosine
// coefficients.  Each item rewrites its own two bins, so no barrier is needed
// between reading and writing.
template <typename T, int LOGN, int BC, int NREG>
__device__ __forceinline__ void cols_apply_symbol(cplx<T> *buf, int job0, int njobs, const Slot &s,
                                                  const cplx<T> *__restrict__ twd) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int IPT = pair_items_per_thread<LOGN, NREG>();
    const double invN2 = 1.0 / ((double)N * (double)N);
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NT;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        if (reg >= njobs) continue;
        const int job = job0 + reg;
        const int c = job / H, j = job % H;
        const double al = s.alpha[c], be = s.beta[c];
        cplx<T> *z = buf + reg * N;
        const int nl = (l == 0) ? H : N - l;
        const cplx<T> zl = z[l], zn = z[nl];
        if constexpr (BC == BC_P) {
            if (j > 0) {
                const T m1 = (T)symbol_mult(s.eig, j, l, al, be, invN2);
                const T m2 = (T)symbol_mult(s.eig, j, nl, al, be, invN2);
                z[l] = {zl.re * m1, zl.im * m1};
                z[nl] = {zn.re * m2, zn.im * m2};
            } else if (l == 0) {
                // bins 0 and N/2 of the packed (kx = 0, kx = N/2) column: real pairs
                z[0] = {zl.re * (T)symbol_mult(s.eig, 0, 0, al, be, invN2),
                        zl.im * (T)symbol_mult(s.eig, H, 0, al, be, invN2)};
                z[H] = {zn.re * (T)symbol_mult(s.eig, 0, H, al, be, invN2),
                        zn.im * (T)symbol_mult(s.eig, H, H, al, be, invN2)};
            } else {
                const T ma = (T)symbol_mult(s.eig, 0, l, al, be, invN2);
                const T mb = (T)symbol_mult(s.eig, H, l, al, be, invN2);
                cplx<T> A = {(zl.re + zn.re) * (T)0.5, (zl.im - zn.im) * (T)0.5};
                cplx<T> B = {(zl.im + zn.im) * (T)0.5, (zn.re - zl.re) * (T)0.5};
                A = {A.re * ma, A.im * ma};
                B = {B.re * mb, B.im * mb};
                z[l] = {A.re - B.im, A.im + B.re};
                z[nl] = {A.re + B.im, B.re - A.im};
            }
        } else {
            const int ka = 2 * j, kb = 2 * j + 1;
            if (l == 0) {
                z[0] = {zl.re * (T)symbol_mult(s.eig, ka, 0, al, be, invN2),
                        zl.im * (T)symbol_mult(s.eig, kb, 0, al, be, invN2)};
                z[H] = {zn.re * (T)symbol_mult(s.eig, ka, H, al, be, invN2),
                        zn.im * (T)symbol_mult(s.eig, kb, H, al, be, invN2)};
            } else {
                const cplx<T> w = twd[l];
                const cplx<T> A = {(zl.re + zn.re) * (T)0.5, (zl.im - zn.im) * (T)0.5};
                const cplx<T> B = {(zl.im + zn.im) * (T)0.5, (zn.re - zl.re) * (T)0.5};
                const cplx<T> qa = cmul(A, w), qb = cmul(B, w);
                // cosine coefficients at l and N-l, scaled by their symbols
                const T xal = qa.re * (T)symbol_mult(s.eig, ka, l, al, be, invN2);
                const T xan = -qa.im * (T)symbol_mult(s.eig, ka, N - l, al, be, invN2);
                const T xbl = qb.re * (T)symbol_mult(s.eig, kb, l, al, be, invN2);
                const T xbn = -qb.im * (T)symbol_mult(s.eig, kb, N - l, al, be, invN2);
                const cplx<T> wc = cconj(w);
                const cplx<T> va = cmul(wc, cplx<T>{xal, -xan});
                const cplx<T> vb = cmul(wc, cplx<T>{xbl, -xbn});
                z[l] = {va.re - vb.im, va.im + vb.re};
                z[nl] = {va.re + vb.im, vb.re - va.im};
            }
        }
    }
    __syncthreads();
}

}  // namespace rdk
