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
// The complex FFTs themselves are in fft16.h (radix-16 Stockham passes in LDS);
// forward sign -1, both directions unnormalised; the 1/N^2 of the 2-D inverse is
// folded into the symbol multiplier.  This file holds the small DFT kernels and
// the pair / cosine pre- and post-processing over padded LDS regions.
#pragma once
#include "rd_dev.h"

namespace rdk {

__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }
template <int LOGN> __host__ __device__ constexpr int lds_region() { return (1 << LOGN) + (1 << LOGN) / 16; }

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

// LDS regions hold N complex values with one padding slot per 16 (fft16.h):
// complex element i of region r lives at r * lds_region<LOGN>() + lds_pad(i).
template <int LOGN> __device__ __forceinline__ int rix(int reg, int i) { return reg * lds_region<LOGN>() + lds_pad(i); }

// Real element m (< 2N) of a region viewed as 2N reals (re, im interleaved).
template <typename T, int LOGN> __device__ __forceinline__ T &rreal(cplx<T> *buf, int reg, int m) {
    return reinterpret_cast<T *>(&buf[rix<LOGN>(reg, m >> 1)])[m & 1];
}

// Work items for the pair steps: item (region, l), l < N/2, owns bins l and N-l
// (item 0 owns bins 0 and N/2).
template <int LOGN, int NREG, int NTH> constexpr int pair_items_per_thread() {
    constexpr int total = NREG * ((1 << LOGN) / 2);
    return (total + NTH - 1) / NTH;
}

// ---- row pass, forward: packed pair spectrum Z -> two rows of slots (in place).
// Periodic: slots of row a hold (A_0, A_{N/2}) then A_1..A_{N/2-1}; row b likewise.
// Neumann: the region, viewed as 2N reals, holds X_a[0..N) then X_b[0..N).
template <typename T, int LOGN, int BC, int NREG, int NTH>
__device__ __forceinline__ void rows_post_forward(cplx<T> *buf, const cplx<T> *__restrict__ twd) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int IPT = pair_items_per_thread<LOGN, NREG, NTH>();
    cplx<T> oa[IPT], ob[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NTH;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        if (l == 0) {
            const cplx<T> z0 = buf[rix<LOGN>(reg, 0)], zh = buf[rix<LOGN>(reg, H)];
            if constexpr (BC == BC_P) {
                oa[i] = {z0.re, zh.re};
                ob[i] = {z0.im, zh.im};
            } else {
                const T s = (T)0.707106781186547524400844362104849039;
                oa[i] = {z0.re, s * zh.re};   // X_a[0], X_a[N/2]
                ob[i] = {z0.im, s * zh.im};
            }
        } else {
            const cplx<T> zl = buf[rix<LOGN>(reg, l)], zn = buf[rix<LOGN>(reg, N - l)];
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
        const int it = threadIdx.x + i * NTH;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        if constexpr (BC == BC_P) {
            buf[rix<LOGN>(reg, l)] = oa[i];
            buf[rix<LOGN>(reg, H + l)] = ob[i];
        } else {
            if (l == 0) {
                rreal<T, LOGN>(buf, reg, 0) = oa[i].re;
                rreal<T, LOGN>(buf, reg, H) = oa[i].im;
                rreal<T, LOGN>(buf, reg, N) = ob[i].re;
                rreal<T, LOGN>(buf, reg, N + H) = ob[i].im;
            } else {
                rreal<T, LOGN>(buf, reg, l) = oa[i].re;
                rreal<T, LOGN>(buf, reg, N - l) = oa[i].im;
                rreal<T, LOGN>(buf, reg, N + l) = ob[i].re;
                rreal<T, LOGN>(buf, reg, 2 * N - l) = ob[i].im;
            }
        }
    }
    __syncthreads();
}

// ---- row pass, inverse: two rows of slots -> packed pair spectrum Z (in place).
template <typename T, int LOGN, int BC, int NREG, int NTH>
__device__ __forceinline__ void rows_pre_inverse(cplx<T> *buf, const cplx<T> *__restrict__ twd) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int IPT = pair_items_per_thread<LOGN, NREG, NTH>();
    cplx<T> zl_out[IPT], zn_out[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NTH;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        if constexpr (BC == BC_P) {
            const cplx<T> a = buf[rix<LOGN>(reg, l)], b = buf[rix<LOGN>(reg, H + l)];
            if (l == 0) {
                zl_out[i] = {a.re, b.re};   // Z_0 = A_0 + i B_0
                zn_out[i] = {a.im, b.im};   // Z_{N/2}
            } else {
                zl_out[i] = {a.re - b.im, a.im + b.re};
                zn_out[i] = {a.re + b.im, b.re - a.im};
            }
        } else {
            if (l == 0) {
                const T r2 = (T)1.41421356237309504880168872420969808;
                zl_out[i] = {rreal<T, LOGN>(buf, reg, 0), rreal<T, LOGN>(buf, reg, N)};
                zn_out[i] = {r2 * rreal<T, LOGN>(buf, reg, H), r2 * rreal<T, LOGN>(buf, reg, N + H)};
            } else {
                const cplx<T> wc = cconj(twd[l]);
                const cplx<T> va = cmul(wc, cplx<T>{rreal<T, LOGN>(buf, reg, l), -rreal<T, LOGN>(buf, reg, N - l)});
                const cplx<T> vb =
                    cmul(wc, cplx<T>{rreal<T, LOGN>(buf, reg, N + l), -rreal<T, LOGN>(buf, reg, 2 * N - l)});
                zl_out[i] = {va.re - vb.im, va.im + vb.re};
                zn_out[i] = {va.re + vb.im, vb.re - va.im};
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NTH;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        buf[rix<LOGN>(reg, l)] = zl_out[i];
        buf[rix<LOGN>(reg, l == 0 ? H : N - l)] = zn_out[i];
    }
    __syncthreads();
}

// Symbol multiplier 1 / (N^2 g), g = (1 + alpha mu + beta mu^2 + gamma mu^3)^2,
// mu = s_kx + s_ky.
__device__ __forceinline__ double symbol_mult(const double *__restrict__ eig, int kx, int ky, double alpha,
                                              double beta, double gamma, double invN2) {
    const double mu = eig[kx] + eig[ky];
    const double a = 1.0 + mu * (alpha + mu * (beta + gamma * mu));
    return invN2 / (a * a);
}

// ---- column pass, between the forward and inverse column FFTs: multiply by the
// symbol.  Region `reg` holds column job (component c, column j) with
// c = job / H, j = job % H.  Periodic: column j is the row spectrum at kx = j;
// column 0 packs kx = 0 (real part) and kx = N/2 (imaginary part).  Neumann:
// column j packs kx = 2j (real) and kx = 2j + 1 (imaginary), both cosine
// coefficients.  Each item rewrites its own two bins, so no barrier is needed
// between reading and writing.
template <typename T, int LOGN, int BC, int NREG, int NTH>
__device__ __forceinline__ void cols_apply_symbol(cplx<T> *buf, int job0, int njobs, SlotRef s,
                                                  const cplx<T> *__restrict__ twd) {
    constexpr int N = 1 << LOGN, H = N / 2;
    constexpr int IPT = pair_items_per_thread<LOGN, NREG, NTH>();
    const double invN2 = 1.0 / ((double)N * (double)N);
    // FP32: not unrolled, which keeps the FP32 column pass within 128 registers
    // (no spills) so that two of its workgroups fit on a compute unit
    constexpr int UNR = sizeof(T) == 4 ? 1 : IPT;
#pragma unroll UNR
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + i * NTH;
        if (it >= NREG * H) break;
        const int reg = it / H, l = it % H;
        if (reg >= njobs) continue;
        const int job = job0 + reg;
        const int c = job / H, j = job % H;
        const double al = s.alpha[c], be = s.beta[c], ga = s.gamma[c];
        const int nl = (l == 0) ? H : N - l;
        cplx<T> &zlr = buf[rix<LOGN>(reg, l)];
        cplx<T> &znr = buf[rix<LOGN>(reg, nl)];
        const cplx<T> zl = zlr, zn = znr;
        if constexpr (BC == BC_P) {
            if (j > 0) {
                const T m1 = (T)symbol_mult(s.eig, j, l, al, be, ga, invN2);
                const T m2 = (T)symbol_mult(s.eig, j, nl, al, be, ga, invN2);
                zlr = {zl.re * m1, zl.im * m1};
                znr = {zn.re * m2, zn.im * m2};
            } else if (l == 0) {
                // bins 0 and N/2 of the packed (kx = 0, kx = N/2) column: real pairs
                zlr = {zl.re * (T)symbol_mult(s.eig, 0, 0, al, be, ga, invN2),
                       zl.im * (T)symbol_mult(s.eig, H, 0, al, be, ga, invN2)};
                znr = {zn.re * (T)symbol_mult(s.eig, 0, H, al, be, ga, invN2),
                       zn.im * (T)symbol_mult(s.eig, H, H, al, be, ga, invN2)};
            } else {
                const T ma = (T)symbol_mult(s.eig, 0, l, al, be, ga, invN2);
                const T mb = (T)symbol_mult(s.eig, H, l, al, be, ga, invN2);
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
                zlr = {zl.re * (T)symbol_mult(s.eig, ka, 0, al, be, ga, invN2),
                       zl.im * (T)symbol_mult(s.eig, kb, 0, al, be, ga, invN2)};
                znr = {zn.re * (T)symbol_mult(s.eig, ka, H, al, be, ga, invN2),
                       zn.im * (T)symbol_mult(s.eig, kb, H, al, be, ga, invN2)};
            } else {
                const cplx<T> w = twd[l];
                const cplx<T> A = {(zl.re + zn.re) * (T)0.5, (zl.im - zn.im) * (T)0.5};
                const cplx<T> B = {(zl.im + zn.im) * (T)0.5, (zn.re - zl.re) * (T)0.5};
                const cplx<T> qa = cmul(A, w), qb = cmul(B, w);
                // cosine coefficients at l and N-l, scaled by their symbols
                const T xal = qa.re * (T)symbol_mult(s.eig, ka, l, al, be, ga, invN2);
                const T xan = -qa.im * (T)symbol_mult(s.eig, ka, N - l, al, be, ga, invN2);
                const T xbl = qb.re * (T)symbol_mult(s.eig, kb, l, al, be, ga, invN2);
                const T xbn = -qb.im * (T)symbol_mult(s.eig, kb, N - l, al, be, ga, invN2);
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

}  // namespace rdk
