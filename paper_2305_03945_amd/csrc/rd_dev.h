// Device-side data structures shared by the HIP kernels and the host runtime.
//
// A "slot" is one implicit-step problem resident on the GPU: its parameters,
// its workspace pointers and its iteration state.  Every kernel takes an array
// of slot pointers and processes slot blockIdx.y, so a single step (rd_step) and
// a batch of same-shape steps of different trajectories (serving) run the same
// kernels.  All slots of one launch share N, dimension, boundary condition,
// equation family and precision (these are template parameters, or select the
// kernel); everything else is per slot.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

template <typename T> struct cplx { T re, im; };

// Per-slot iteration state, written only by k_finalize (after the fixed-order
// reduction of a residual pass) and read at the start of every kernel.
struct State {
    int done;          // inner loop finished (FP64 path: the whole step)
    int iters;         // iterations of the current (inner) PDHG loop
    int total_iters;   // mixed: inner iterations summed over outer passes
    int outer;         // mixed: outer passes completed
    int outer_done;    // mixed: step finished
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

// ---------------------------------------------------------------- address spaces
// Slots and their States are read through the constant address space: the
// fields are uniform across a workgroup, so they become scalar loads.  A kernel
// never writes the slot it reads this way (State is written only by thread 0 of
// k_finalize, through a plain pointer), and scalar caches are invalidated at
// every kernel start, so the values seen are those of the previous launch.
typedef const __attribute__((address_space(4))) Slot &SlotRef;
typedef const __attribute__((address_space(4))) State &StateRef;
__device__ __forceinline__ SlotRef slot_ref(const Slot *p) {
    return *(const __attribute__((address_space(4))) Slot *)p;
}
__device__ __forceinline__ SlotRef slot_of(Slot *const *slots) { return slot_ref(slots[blockIdx.y]); }
__device__ __forceinline__ StateRef state_of(SlotRef s) {
    return *(const __attribute__((address_space(4))) State *)s.st;
}

// Buffers are addressed through the global address space: pointers loaded from
// memory are otherwise generic, and generic (flat) accesses are slower.
template <typename T> using gptr_t = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gptr_t<T> gp(T *p) { return (gptr_t<T>)p; }

// ---------------------------------------------------------------- XCD-aware tiling
// The MI355X dispatches workgroups to its 8 XCDs round-robin by linear id, and
// each XCD has its own L2.  Kernels whose tiles read halo rows of their
// neighbours map workgroup b to tile (b % 8) * (nb / 8) + b / 8, so that every
// XCD sweeps one contiguous band of the grid and the halo rows it re-reads are
// in its own L2.  (Identity when nb is not a multiple of 8.)
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    return (nb % NXCD) ? b : (b % NXCD) * (nb / NXCD) + b / NXCD;
}

// ---------------------------------------------------------------- small helpers
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename T> __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.re, -a.im}; }

// Ghost-cell index maps.  Periodic: wrap.  Neumann: half-sample mirror
// (index -1-m -> m, N+m -> N-1-m), valid for offsets up to N.
template <int BC> __device__ __forceinline__ int wrap(int i, int N) {
    if (BC == BC_P) return i & (N - 1);
    if (i < 0) return -1 - i;
    if (i >= N) return 2 * N - 1 - i;
    return i;
}

// Position of x in the Makhoul even/odd reordering used for the DCT-II:
// x = 2n -> n, x = 2n + 1 -> N - 1 - n.
__device__ __forceinline__ int dct_pos(int x, int N) { return (x & 1) ? (N - 1 - (x >> 1)) : (x >> 1); }

// Rows of the grid one row-pass workgroup owns.  The workgroup's NT threads
// form NT / (N/16) transform teams (one transform per N/16 threads); a row
// pair is one transform, so R = 2 * teams keeps every team busy (R N = 32 NT
// reals of LDS per component).  At least 2, at most N/4 (so that every grid
// spans at least four workgroups), and for two components at most half that.
// Where one team spans the workgroup (N >= 16 NT), FP32 workgroups take two
// row pairs, transformed in turn, so that the spectrum tiles are four rows high
// and the column pass reads 128-byte runs.  This is the row count of the 3-D
// row passes.
template <typename T, int LOGN, int C> constexpr int rows_per_block3() {
    constexpr int N = 1 << LOGN;
    constexpr int teams = (N / 16 >= NT) ? 1 : NT / (N / 16);
    constexpr int pairs = (N / 16 >= NT && sizeof(T) == 4) ? 2 : 1;
    constexpr int want = 2 * teams * pairs / C;
    constexpr int cap = N / 4;
    constexpr int r = want < 2 ? 2 : (want > cap ? cap : want);
    return r;
}

// 2-D row passes: below 2048^2 the rule above leaves few workgroups (N = 128:
// 4 of 32 rows, N = 512: 32 of 16), and a pass waits on their serial stencil
// loops while most CUs idle.  At most N/256 rows (at least 2: N/2 workgroups
// up to N = 512, 256 at N = 1024) leave transform teams idle instead and are
// faster on every grid measured (steps, ms: 128^2 FCH 7.9 -> 6.6, 256^2
// Allen-Cahn 0.84 -> 0.63, 256^2 Neumann Cahn-Hilliard 1.04 -> 0.69, 512^2
// 1.07 -> 0.82, 1024^2 1.39 -> 1.25; N/32, N/64 and N/128 rows measured in
// between).  2048^2 and 4096^2 keep 4 rows.  The 3-D row passes keep theirs:
// there the stop decision reduces one partial sum per workgroup of N^2 / R,
// and more of them slowed the y pass that takes it.
template <typename T, int LOGN, int C> constexpr int rows_per_block() {
    constexpr int N = 1 << LOGN;
    constexpr int r3 = rows_per_block3<T, LOGN, C>();
    constexpr int small = N / 256 < 2 ? 2 : N / 256;
    return r3 < small ? r3 : small;
}

}  // namespace rdk
