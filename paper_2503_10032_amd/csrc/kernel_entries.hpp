// Template kernels compiled in translation units of their own, so that the
// library's device code builds in parallel: the Householder panel kernel for
// each rows-per-thread count (inst_qr_panel_*.hip) and the persistent CG
// kernel for each right-hand-side width (inst_cg_fused_*.hip).  The main unit
// reaches them only through these functions.
#pragma once
#include <hip/hip_runtime.h>

namespace ddelm {

struct QRDesc;

// k_qr_panel16<T, RPT, NT> on `grid` workgroups of NT threads.
template <typename T, int RPT, int NT>
void launch_qr_panel16_rpt(dim3 grid, hipStream_t s, const QRDesc* d, T* A, T* tau, T* Tb, int k, int panel,
                           int npanel);

// Address of k_cg_fused<T, NR> (for attributes, occupancy and the cooperative launch).
template <typename T, int NR>
const void* cg_fused_kernel();

}  // namespace ddelm
