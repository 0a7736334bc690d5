// Instantiates every FFT-carrying kernel for one grid size N = 2^RD_LOGN (set by
// the build) and registers the launchers.
#include "kernels.h"
#include "kernels3d.h"
#include "kernels_wg.h"
#include "registry.h"

#include <hip/hip_ext.h>

#ifndef RD_LOGN
#error "RD_LOGN must be defined by the build"
#endif

namespace rdk {
namespace {

constexpr int L = RD_LOGN;

template <int EQ> constexpr int ncomp() { return EQ == EQ_SCHNAK ? 2 : 1; }

inline hipEvent_t ev_start(hipEvent_t *ev) { return ev ? ev[0] : nullptr; }
inline hipEvent_t ev_stop(hipEvent_t *ev) { return ev ? ev[1] : nullptr; }

template <typename T, int EQ> constexpr int row_block() { return rows_per_block<T, L, ncomp<EQ>()>(); }
template <typename T, int EQ> constexpr int row_block3() { return rows_per_block3<T, L, ncomp<EQ>()>(); }

// The row kernel writes per-workgroup partial sums; the stop decision is taken
// by k_finalize (launch_fin) or by the extra workgroup of the next column pass.
template <typename T, int BC, int EQ, int KIND>
void launch_rowfwd(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    constexpr int R = row_block<T, EQ>();
    hipExtLaunchKernelGGL((k_row_forward<T, L, BC, EQ, KIND>), dim3((1 << L) / R, nslots), dim3(NT), 0, st,
                          ev_start(ev), ev_stop(ev), 0, slots);
}

template <int KIND, int EQ>
void launch_fin(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    hipExtLaunchKernelGGL((k_finalize<KIND, ncomp<EQ>()>), dim3(1, nslots), dim3(NT), 0, st, ev_start(ev),
                          ev_stop(ev), 0, slots);
}

// Initial pass: row kernel, then its decision at once.
template <typename T, int BC, int EQ, int KIND>
void launch_rowfwd_fin(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    hipEvent_t e0[2] = {ev_start(ev), nullptr}, e1[2] = {nullptr, ev_stop(ev)};
    launch_rowfwd<T, BC, EQ, KIND>(slots, nslots, st, e0);
    launch_fin<KIND, EQ>(slots, nslots, st, e1);
}

template <typename T, int BC, int EQ, int FIN>
void launch_cols(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    constexpr int jobs = ncomp<EQ>() * (1 << L) / 2;
    constexpr int CB = col_jobs<T, L, ncomp<EQ>()>();
    static_assert(((1 << L) / 2) % CB == 0, "column blocks must tile a component");
    constexpr int extra = FIN == FIN_NONE ? 0 : 1;
    hipExtLaunchKernelGGL((k_cols<T, L, BC, ncomp<EQ>(), FIN>), dim3(jobs / CB + extra, nslots),
                          dim3(col_threads<T, L, ncomp<EQ>()>()), 0, st, ev_start(ev), ev_stop(ev), 0, slots);
}

template <typename T, int BC, int EQ>
void launch_rowinv(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    constexpr int R = row_block<T, EQ>();
    hipExtLaunchKernelGGL((k_rowinv<T, L, BC, ncomp<EQ>()>), dim3((1 << L) / R, nslots), dim3(NT), 0, st,
                          ev_start(ev), ev_stop(ev), 0, slots);
}

template <typename T, int BC, int EQ, int MODE>
void launch_upd(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    constexpr int blocks = ((1 << L) * (1 << L) / UPD_PPT + NT - 1) / NT;
    hipExtLaunchKernelGGL((k_upd<T, L, BC, EQ, MODE>), dim3(blocks, nslots), dim3(NT), 0, st, ev_start(ev),
                          ev_stop(ev), 0, slots);
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

// Small grids: the whole step in one launch, one workgroup per slot.
template <typename T, int BC, int EQ, int MODE>
void launch_step_wg(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    hipExtLaunchKernelGGL((k_step_wg<T, L, BC, EQ, MODE>), dim3(1, nslots), dim3(NT7), 0, st, ev_start(ev),
                          ev_stop(ev), 0, slots);
}

template <int BC, int EQ> void fill_mixed();

template <int BC, int EQ> void fill() {
    KSet &f = g_kernels[MODE_F64][L][BC][EQ];
    f.init = launch_rowfwd_fin<double, BC, EQ, K_INIT64>;
    f.rowfwd = launch_rowfwd<double, BC, EQ, K_ITER64>;
    f.fin = launch_fin<K_ITER64, EQ>;
    f.cols = launch_cols<double, BC, EQ, FIN_NONE>;
    f.cols_fin = launch_cols<double, BC, EQ, K_ITER64>;
    f.rowinv = launch_rowinv<double, BC, EQ>;
    f.upd = launch_upd<double, BC, EQ, MODE_F64>;
    f.tin = launch_tin<double, BC, EQ>;
    f.tout = launch_tout<double, BC, EQ>;
    f.rows_per_block = row_block<double, EQ>();
    if constexpr (wg_step_available<double, L, EQ>()) f.step_wg = launch_step_wg<double, BC, EQ, MODE_F64>;
    fill_mixed<BC, EQ>();
}

template <int BC, int EQ> void fill_mixed() {
    KSet &m = g_kernels[MODE_MIXED][L][BC][EQ];
    m.init = launch_rowfwd_fin<float, BC, EQ, K_OUTER_INIT>;
    // the iteration row pass makes the outer update itself when the inner loop
    // has stopped, and the decisions after it follow (no separate outer launch)
    m.rowfwd = launch_rowfwd<float, BC, EQ, K_MIXED>;
    m.fin = launch_fin<K_MIXED, EQ>;
    m.cols = launch_cols<float, BC, EQ, FIN_NONE>;
    m.cols_fin = launch_cols<float, BC, EQ, K_MIXED>;
    m.rowinv = launch_rowinv<float, BC, EQ>;
    m.upd = launch_upd<float, BC, EQ, MODE_MIXED>;
    m.tin = launch_tin<float, BC, EQ>;
    m.tout = launch_tout<float, BC, EQ>;
    m.rows_per_block = row_block<float, EQ>();
    if constexpr (wg_step_available<float, L, EQ>()) m.step_wg = launch_step_wg<float, BC, EQ, MODE_MIXED>;
}

// ---------------------------------------------------------------- 3-D launchers
template <typename T, int BC, int EQ, int KIND>
void launch3_rowfwd_fin(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    constexpr int R = row_block3<T, EQ>();
    constexpr int N = 1 << L;
    hipExtLaunchKernelGGL((k3_row_forward<T, L, BC, EQ, KIND>), dim3(N * (N / R), nslots), dim3(NT), 0, st,
                          ev_start(ev), nullptr, 0, slots);
    hipExtLaunchKernelGGL((k_finalize<KIND, ncomp<EQ>()>), dim3(1, nslots), dim3(NT), 0, st, nullptr, ev_stop(ev), 0,
                          slots);
}

template <typename T, int BC, int EQ, int PASS, int FIN>
void launch3_lines(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    constexpr int N = 1 << L;
    constexpr int CB = line_cb<T, L>();
    static_assert((N / 2) % CB == 0, "line blocks must tile the slots");
    constexpr int extra = FIN == FIN_NONE ? 0 : 1;
    hipExtLaunchKernelGGL((k3_lines<T, L, BC, ncomp<EQ>(), PASS, FIN>),
                          dim3(ncomp<EQ>() * N * ((N / 2) / CB) + extra, nslots), dim3(line_threads<T, L>()), 0, st,
                          ev_start(ev), ev_stop(ev), 0, slots);
}

template <typename T, int BC, int EQ, int KIND>
void launch3_rowfwd(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    constexpr int R = row_block3<T, EQ>();
    constexpr int N = 1 << L;
    hipExtLaunchKernelGGL((k3_row_forward<T, L, BC, EQ, KIND>), dim3(N * (N / R), nslots), dim3(NT), 0, st,
                          ev_start(ev), ev_stop(ev), 0, slots);
}

template <typename T, int BC, int EQ>
void launch3_rowinv(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    constexpr int R = row_block3<T, EQ>();
    constexpr int N = 1 << L;
    hipExtLaunchKernelGGL((k3_rowinv<T, L, BC, ncomp<EQ>()>), dim3(N * (N / R), nslots), dim3(NT), 0, st,
                          ev_start(ev), ev_stop(ev), 0, slots);
}

template <typename T, int BC, int EQ, int MODE>
void launch3_upd(Slot *const *slots, int nslots, hipStream_t st, hipEvent_t *ev) {
    hipExtLaunchKernelGGL((k3_upd<T, L, BC, EQ, MODE>), dim3(upd3_blocks<T, L>(), nslots), dim3(NT), 0, st,
                          ev_start(ev), ev_stop(ev), 0, slots);
}

template <typename T, int BC, int EQ>
void launch3_tin(Slot *const *slots, int nslots, const double *in, double *, hipStream_t st) {
    constexpr int R = row_block3<T, EQ>();
    constexpr int N = 1 << L;
    hipLaunchKernelGGL((k3_rows_transform_in<T, L, BC, ncomp<EQ>()>), dim3(N * (N / R), nslots), dim3(NT), 0, st,
                       slots, in);
}

template <typename T, int BC, int EQ>
void launch3_tout(Slot *const *slots, int nslots, const double *, double *out, hipStream_t st) {
    constexpr int R = row_block3<T, EQ>();
    constexpr int N = 1 << L;
    hipLaunchKernelGGL((k3_rows_transform_out<T, L, BC, ncomp<EQ>()>), dim3(N * (N / R), nslots), dim3(NT), 0, st,
                       slots, out);
}

template <typename T, int BC, int EQ, int MODE> void fill3_mode(KSet &k) {
    constexpr bool f64 = MODE == MODE_F64;
    // mixed: the row pass makes the outer update itself (as in 2-D)
    constexpr int KIT = f64 ? K_ITER64 : K_MIXED;
    k.init = launch3_rowfwd_fin<T, BC, EQ, f64 ? K_INIT64 : K_OUTER_INIT>;
    k.rowfwd = launch3_rowfwd<T, BC, EQ, KIT>;
    k.fin = launch_fin<KIT, EQ>;
    k.yfwd = launch3_lines<T, BC, EQ, L3_YFWD, FIN_NONE>;
    k.yfwd_fin = launch3_lines<T, BC, EQ, L3_YFWD, KIT>;
    k.zsym = launch3_lines<T, BC, EQ, L3_ZSYM, FIN_NONE>;
    k.yinv = launch3_lines<T, BC, EQ, L3_YINV, FIN_NONE>;
    k.rowinv = launch3_rowinv<T, BC, EQ>;
    k.upd = launch3_upd<T, BC, EQ, MODE>;
    k.tin = launch3_tin<T, BC, EQ>;
    k.tout = launch3_tout<T, BC, EQ>;
    k.rows_per_block = row_block3<T, EQ>();
    k.dim = 3;
}

template <int BC, int EQ> void fill3() {
    if constexpr (L <= LOGN3_MAX) {
        fill3_mode<double, BC, EQ, MODE_F64>(g_kernels3[MODE_F64][L][BC][EQ]);
        fill3_mode<float, BC, EQ, MODE_MIXED>(g_kernels3[MODE_MIXED][L][BC][EQ]);
    }
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
    fill<BC_P, EQ_FCH>();
    fill<BC_N, EQ_FCH>();
    fill3<BC_P, EQ_LAP5>();
    fill3<BC_P, EQ_SCHNAK>();
    fill3<BC_N, EQ_LAP5>();
    fill3<BC_N, EQ_SCHNAK>();
}

}  // namespace rdk
