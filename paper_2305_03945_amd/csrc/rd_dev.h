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

#include "rd_types.h"

namespace rdk {

template <typename T> struct cplx { T re, im; };

// ---------------------------------------------------------------- address spaces
// Slots are read through the constant address space: the fields are uniform
// across a workgroup, so they become scalar loads.  The host writes a slot
// before the launches that read it and no kernel writes one.
typedef const __attribute__((address_space(4))) Slot &SlotRef;
__device__ __forceinline__ SlotRef slot_ref(const Slot *p) {
    return *(const __attribute__((address_space(4))) Slot *)p;
}
__device__ __forceinline__ SlotRef slot_of(Slot *const *slots) { return slot_ref(slots[blockIdx.y]); }

// ---------------------------------------------------------------- the State, read coherently
// The State is written by the stop decision of one launch and read by the
// following launches (and, in a column pass or forward y pass, by the other
// workgroups of the deciding launch itself).  Every read is a relaxed atomic
// load at agent scope: a vector load that bypasses the non-coherent caches
// (the per-CU vector L1 and the scalar cache), so its value never depends on
// whether those caches were invalidated when the kernel was dispatched.
template <typename X> __device__ __forceinline__ X ld_agent(const X *p) {
    return __hip_atomic_load((const __attribute__((address_space(1))) X *)p, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

struct StateV {
    int done, iters, outer, outer_done;
};
// The four fields that select what a launch does, read once per workgroup (two
// 8-byte loads by thread 0; one request per workgroup rather than per wave keeps
// the thousands of workgroups of a launch from queueing on the one line) and
// handed to every thread through LDS.  Called by every thread of the workgroup,
// before any thread leaves the kernel.
__device__ __forceinline__ StateV state_of(SlotRef s) {
    __shared__ unsigned long long sh_state[2];
    if (threadIdx.x == 0) {
        const unsigned long long *p = (const unsigned long long *)s.st;
        sh_state[0] = ld_agent(p);
        sh_state[1] = ld_agent(p + 1);
    }
    __syncthreads();
    const unsigned long long a = sh_state[0], b = sh_state[1];
    StateV v;
    v.done = __builtin_amdgcn_readfirstlane((int)(unsigned)(a & 0xffffffffu));
    v.iters = __builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
    v.outer = __builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xffffffffu));
    v.outer_done = __builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return v;
}
typedef const StateV &StateRef;

// The whole State, for the stop decision (one thread).
__device__ __forceinline__ State load_state(const State *st) {
    State v;
    v.done = ld_agent(&st->done);
    v.iters = ld_agent(&st->iters);
    v.total_iters = ld_agent(&st->total_iters);
    v.outer = ld_agent(&st->outer);
    v.outer_done = ld_agent(&st->outer_done);
    v.status = ld_agent(&st->status);
    v.inner_best_it = ld_agent(&st->inner_best_it);
    v.pad = 0;
    v.res = ld_agent(&st->res);
    v.res0 = ld_agent(&st->res0);
    v.outer_res = ld_agent(&st->outer_res);
    v.inner_target = ld_agent(&st->inner_target);
    v.mass = ld_agent(&st->mass);
    v.inner_res = ld_agent(&st->inner_res);
    v.inner_best = ld_agent(&st->inner_best);
    return v;
}
template <typename X> __device__ __forceinline__ void st_agent(X *p, X v) {
    __hip_atomic_store((__attribute__((address_space(1))) X *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Stores the decided State; the release fence makes it visible device-wide
// before the kernel ends.
__device__ __forceinline__ void store_state(State *st, const State &v) {
    st_agent(&st->done, v.done);
    st_agent(&st->iters, v.iters);
    st_agent(&st->total_iters, v.total_iters);
    st_agent(&st->outer, v.outer);
    st_agent(&st->outer_done, v.outer_done);
    st_agent(&st->status, v.status);
    st_agent(&st->inner_best_it, v.inner_best_it);
    st_agent(&st->res, v.res);
    st_agent(&st->res0, v.res0);
    st_agent(&st->outer_res, v.outer_res);
    st_agent(&st->inner_target, v.inner_target);
    st_agent(&st->mass, v.mass);
    st_agent(&st->inner_res, v.inner_res);
    st_agent(&st->inner_best, v.inner_best);
    __threadfence();
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
