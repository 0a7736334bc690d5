// Host-side tables of kernel launchers (2-D grids, and 3-D grids for log2 N <=
// LOGN3_MAX), one entry per (precision mode, log2 N, boundary condition, equation
// family).  Each instantiation unit fills the entries of one log2 N; the
// size-independent kernels fill their own fields.
#pragma once
#include <hip/hip_runtime.h>
#include "rd_types.h"

namespace rdk {

// ev: nullptr, or {start, stop} events that the dispatch packets of the launch
// record (start of its first kernel, end of its last), for kernel timing.
typedef void (*launch_fn)(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev);
typedef void (*launch_io_fn)(Slot *const *slots, int nslots, const double *in, double *out, hipStream_t st);

struct KSet {
    launch_fn init = nullptr;       // FP64: K_INIT64; mixed: K_OUTER_INIT
    launch_fn cols = nullptr;       // column pass (T)
    launch_fn cols_fin = nullptr;   // column pass + stop decision of the preceding iteration row pass
    launch_fn fin = nullptr;        // stop decision of an iteration row pass (k_finalize)
    launch_fn rowinv = nullptr;     // inverse rows + dual update (T)
    launch_fn upd = nullptr;        // primal update (T)
    launch_fn rowfwd = nullptr;     // FP64: K_ITER64; mixed: K_MIXED (inner or outer pass); no decision
    launch_fn step_wg = nullptr;    // small grids: the whole step, one workgroup per slot (k_step_wg)
    launch_fn yfwd = nullptr;       // 3-D: forward y-transforms
    launch_fn yfwd_fin = nullptr;   // 3-D: the same, plus the stop decision of the preceding row pass
    launch_fn zsym = nullptr;       // 3-D: forward z-transform, symbol, inverse z-transform
    launch_fn yinv = nullptr;       // 3-D: inverse y-transforms
    launch_io_fn tin = nullptr;     // precond-only: FP64 W -> row transforms into S
    launch_io_fn tout = nullptr;    // precond-only: S -> inverse rows -> FP64 Y
    int rows_per_block = 0;
    int dim = 2;                    // 3: the 3-D launch sequence (line passes between the row passes)
};

constexpr int LOGN_MIN = 4, LOGN_MAX = 12;
constexpr int LOGN3_MAX = 8;   // 3-D grids: N <= 256
extern KSet g_kernels[2][LOGN_MAX + 1][2][EQ_COUNT];
extern KSet g_kernels3[2][LOGN3_MAX + 1][2][EQ_COUNT];

void register_upd_kernels();
#define RD_DECLARE_LOGN(L) void register_logn_##L();
RD_DECLARE_LOGN(4) RD_DECLARE_LOGN(5) RD_DECLARE_LOGN(6) RD_DECLARE_LOGN(7) RD_DECLARE_LOGN(8)
RD_DECLARE_LOGN(9) RD_DECLARE_LOGN(10) RD_DECLARE_LOGN(11) RD_DECLARE_LOGN(12)
#undef RD_DECLARE_LOGN

// Bytes of the device scratch array behind rd_step_noalloc, and its device address
// on the current device (hipGetSymbolAddress; call once per device, that device
// current).
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
hipError_t noalloc_scratch_address(void **out);

// Size-independent single-slot kernels used by the kernel-level entry points.
void launch_residual(int bc, int eq, const Slot *slot_dev, int N, const double *U, const double *Uk, double *W,
                     double *partials, hipStream_t st);
void launch_prox(int eq, const Slot *slot_dev, int N, const double *c, double *u, hipStream_t st);
// Copy of a finished step's result (n doubles, n % 4 == 0) to out; a no-op while
// the slot's step runs.
void launch_copy_out(Slot *const *slots, double *out, size_t n, hipStream_t st);
// Serving: each finished slot's result (n doubles, n % 4 == 0) to its src buffer.
void launch_copy_back(Slot *const *slots, int nslots, size_t n, hipStream_t st);

}  // namespace rdk
