// The kernel table and the size-independent single-slot kernels (residual and
// prox) of the kernel-level entry points.
#include "kernels.h"
#include "registry.h"

namespace rdk {

KSet g_kernels[2][LOGN_MAX + 1][2][EQ_COUNT];
KSet g_kernels3[2][LOGN3_MAX + 1][2][EQ_COUNT];

// Workspace of rd_step_noalloc: every buffer its kernels use (slot, State, partial
// sums, tables, iterate fields) is carved from this array, so that the entry point
// allocates nothing.  Each device the library runs on holds its own copy for the
// life of the process.  In host code the name is not a device address: host code
// uses only the address noalloc_scratch_address() returns for the current device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

hipError_t noalloc_scratch_address(void **out) {
    return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

void launch_residual(int bc, int eq, const Slot *slot_dev, int N, const double *U, const double *Uk, double *W,
                     double *partials, hipStream_t st) {
    const int blocks = (int)(((size_t)N * N + NT - 1) / NT);
    const dim3 g(blocks), b(NT);
#define RD_RES(BCV, EQV) \
    hipLaunchKernelGGL((k_residual<BCV, EQV>), g, b, 0, st, slot_dev, U, Uk, W, partials)
    if (bc == BC_P) {
        if (eq == EQ_LAP5) RD_RES(BC_P, EQ_LAP5);
        else if (eq == EQ_BIH) RD_RES(BC_P, EQ_BIH);
        else if (eq == EQ_FCH) RD_RES(BC_P, EQ_FCH);
        else RD_RES(BC_P, EQ_SCHNAK);
    } else {
        if (eq == EQ_LAP5) RD_RES(BC_N, EQ_LAP5);
        else if (eq == EQ_BIH) RD_RES(BC_N, EQ_BIH);
        else if (eq == EQ_FCH) RD_RES(BC_N, EQ_FCH);
        else RD_RES(BC_N, EQ_SCHNAK);
    }
#undef RD_RES
}

// Result of a finished step -> the caller's buffer (n doubles, n % 4 == 0): the
// FP64 iterate U[iters & 1] or the mixed path's FP64 U64[outer & 1].  Returns at
// once while the step still runs, so the host enqueues it after every chunk of
// iterations and needs no launch of its own once the step has finished; and when
// that buffer is the caller's (the host may bind the output as one of the two).
__global__ __launch_bounds__(NT) void k_copy_out(Slot *const *slots, double *out, size_t n) {
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if (!sst.outer_done) return;
    const double *src = s.mode == MODE_F64 ? (const double *)s.U[sst.iters & 1] : s.U64[sst.outer & 1];
    if (src == out) return;   // the step ended in the caller's buffer
    const auto in4 = gp((const vec4_t<double> *)src);
    const auto out4 = gp((vec4_t<double> *)out);
    for (size_t i = blockIdx.x * (size_t)NT + threadIdx.x; i < n / 4; i += (size_t)gridDim.x * NT) out4[i] = in4[i];
}

void launch_copy_out(Slot *const *slots, double *out, size_t n, hipStream_t st) {
    const size_t want = (n / 4 + NT - 1) / NT;
    const int blocks = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(k_copy_out, dim3(blocks), dim3(NT), 0, st, slots, out, n);
}

// Serving: the steps of a batch of slots (blockIdx.y) that finished with status
// ok replace their trajectories' resident states, which are the steps' inputs
// (src); a slot whose step still runs, or failed (no convergence, not finite), is
// left alone, so that the trajectory keeps U^k.  The input is read only by the
// initial pass, so once the step has finished it may be overwritten.
__global__ __launch_bounds__(NT) void k_copy_back(Slot *const *slots, size_t n) {
    SlotRef s = slot_of(slots);
    StateRef sst = state_of(s);
    if (!sst.outer_done) return;
    __shared__ int sh_status;
    if (threadIdx.x == 0) sh_status = ld_agent(&s.st->status);
    __syncthreads();
    if (sh_status != ST_OK) return;
    const double *src = s.mode == MODE_F64 ? (const double *)s.U[sst.iters & 1] : s.U64[sst.outer & 1];
    const auto in4 = gp((const vec4_t<double> *)src);
    const auto out4 = gp((vec4_t<double> *)const_cast<double *>(s.src));
    for (size_t i = blockIdx.x * (size_t)NT + threadIdx.x; i < n / 4; i += (size_t)gridDim.x * NT) out4[i] = in4[i];
}

void launch_copy_back(Slot *const *slots, int nslots, size_t n, hipStream_t st) {
    const size_t want = (n / 4 + NT - 1) / NT;
    const int blocks = (int)(want < 2048 ? want : 2048);
    hipLaunchKernelGGL(k_copy_back, dim3(blocks, nslots), dim3(NT), 0, st, slots, n);
}

void launch_prox(int eq, const Slot *slot_dev, int N, const double *c, double *u, hipStream_t st) {
    const int blocks = (int)(((size_t)N * N + NT - 1) / NT);
    if (eq == EQ_LAP5) hipLaunchKernelGGL((k_prox<EQ_LAP5>), dim3(blocks), dim3(NT), 0, st, slot_dev, c, u);
    else if (eq == EQ_SCHNAK) hipLaunchKernelGGL((k_prox<EQ_SCHNAK>), dim3(blocks), dim3(NT), 0, st, slot_dev, c, u);
    else hipLaunchKernelGGL((k_prox<EQ_BIH>), dim3(blocks), dim3(NT), 0, st, slot_dev, c, u);
}

}  // namespace rdk
