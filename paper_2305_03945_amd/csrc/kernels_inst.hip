// Instantiates every FFT-carrying kernel for one grid size N = 2^RD_LOGN (set by
// the build) and registers the launchers.
#include "kernels.h"
#include "registry.h"

#ifndef RD_LOGN
#error "RD_LOGN must be defined by the build"
#endif

namespace rdk {
namespace {

constexpr int L = RD_LOGN;

template <int EQ> constexpr int ncomp() { return EQ == EQ_SCHNAK ? 2 : 1; }

template <typename T, int EQ> constexpr int row_block() { return rows_per_block<T, L, ncomp<EQ>()>(); }

// A row-forward pass is two launches: the row kernel writes per-workgroup
// partial sums, k_finalize reduces them and takes the stop decision.
template <typename T, int BC, int EQ, int KIND>
void launch_rowfwd(Slot *const *slots, int nslots, hipStream_t st) {
    constexpr int R = row_block<T, EQ>();
    hipLaunchKernelGGL((k_row_forward<T, L, BC, EQ, KIND>), dim3((1 << L) / R, nslots), dim3(NT), 0, st, slots);
    hipLaunchKernelGGL((k_finalize<KIND, ncomp<EQ>()>), dim3(1, nslots), dim3(NT), 0, st, slots);
}

template <typename T, int BC, int EQ>
void launch_cols(Slot *const *slots, int nslots, hipStream_t st) {
    constexpr int jobs = ncomp<EQ>() * (1 << L) / 2;
    constexpr int CB = col_jobs<T, L, ncomp<EQ>()>();
    static_assert(((1 << L) / 2) % CB == 0, "column blocks must tile a component");
    hipLaunchKernelGGL((k_cols<T, L, BC, ncomp<EQ>()>), dim3(jobs / CB, nslots), dim3(col_threads<T, L, ncomp<EQ>()>()),
                       0, st, slots);
}

template <typename T, int BC, int EQ>
void launch_rowinv(Slot *const *slots, int nslots, hipStream_t st) {
    constexpr int R = row_block<T, EQ>();
    hipLaunchKernelGGL((k_rowinv<T, L, BC, ncomp<EQ>()>), dim3((1 << L) / R, nslots), dim3(NT), 0, st, slots);
}

template <typename T, int BC, int EQ, int MODE>
void launch_upd(Slot *const *slots, int nslots, hipStream_t st) {
    constexpr int blocks = ((1 << L) * (1 << L) / UPD_PPT + NT - 1) / NT;
    hipLaunchKernelGGL((k_upd<T, L, BC, EQ, MODE>), dim3(blocks, nslots), dim3(NT), 0, st, slots);
}

template <typename T, int BC, int EQ>
void launch_tin(Slot *const *slots, int nslots, const double *in, double *, hipStream_t st) {
    constexpr int R = row_block<T, EQ>();
    hipLaunchKernelGGL((k_rows_transform_in<T, L, BC, ncomp<EQ>()>), dim3((1 << L) / R, nslots), dim3(NT), 0, st,
                       slots, in);
}

template <typename T, int BC, int EQ>
void launch_tout(Slot *const *slots, int nslots, const double *, double *out, hipStream_t st) {
    constexpr int R = row_block<T, EQ>();
    hipLaunchKernelGGL((k_rows_transform_out<T, L, BC, ncomp<EQ>()>), dim3((1 << L) / R, nslots), dim3(NT), 0, st,
                       slots, out);
}

template <int BC, int EQ> void fill() {
    KSet &f = g_kernels[MODE_F64][L][BC][EQ];
    f.init = launch_rowfwd<double, BC, EQ, K_INIT64>;
    f.rowfwd = launch_rowfwd<double, BC, EQ, K_ITER64>;
    f.cols = launch_cols<double, BC, EQ>;
    f.rowinv = launch_rowinv<double, BC, EQ>;
    f.upd = launch_upd<double, BC, EQ, MODE_F64>;
    f.tin = launch_tin<double, BC, EQ>;
    f.tout = launch_tout<double, BC, EQ>;
    f.rows_per_block = row_block<double, EQ>();
    KSet &m = g_kernels[MODE_MIXED][L][BC][EQ];
    m.init = launch_rowfwd<float, BC, EQ, K_OUTER_INIT>;
    m.outer = launch_rowfwd<float, BC, EQ, K_OUTER_UPD>;
    m.rowfwd = launch_rowfwd<float, BC, EQ, K_INNER32>;
    m.cols = launch_cols<float, BC, EQ>;
    m.rowinv = launch_rowinv<float, BC, EQ>;
    m.upd = launch_upd<float, BC, EQ, MODE_MIXED>;
    m.tin = launch_tin<float, BC, EQ>;
    m.tout = launch_tout<float, BC, EQ>;
    m.rows_per_block = row_block<float, EQ>();
}

}  // namespace

#define RD_CAT2(a, b) a##b
#define RD_CAT(a, b) RD_CAT2(a, b)
void RD_CAT(register_logn_, RD_LOGN)() {
    fill<BC_P, EQ_LAP5>();
    fill<BC_P, EQ_BIH>();
    fill<BC_P, EQ_SCHNAK>();
    fill<BC_N, EQ_LAP5>();
    fill<BC_N, EQ_BIH>();
    fill<BC_N, EQ_SCHNAK>();
}

}  // namespace rdk
