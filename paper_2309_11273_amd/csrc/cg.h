// Launchers of the static solve and of the implicit (Newmark) step with the
// block-sparse stiffness (cg.hip).
#pragma once

#include "kernels.h"

namespace pdk {

int64_t cg_workspace_doubles(int64_t n_pad);
// K may be null with mf (products by the force kernels, diagonal from the bonds)
hipError_t launch_cg_start(const StepArgs &a, const pd_bsr_dev *K, double *work, int cur, bool mf, hipStream_t s);
// dt > 0: one iteration on the Newmark operator K + (4/dt^2) M; mf: the
// product K p by the double force kernels instead of the stored K
hipError_t launch_cg_iteration(const StepArgs &a, const pd_bsr_dev *K, double *work, double dt, int cur, bool mf,
                               hipStream_t s);
int64_t nm_workspace_doubles(int64_t n_pad);
hipError_t launch_nm_start(const StepArgs &a, const pd_bsr_dev *K, double *work, double dt, int cur, bool mf,
                           hipStream_t s);
hipError_t launch_nm_finish(const StepArgs &a, const pd_bsr_dev *K, double *work, double dt, int cur,
                            hipStream_t s);
hipError_t launch_cg_finish(const StepArgs &a, const pd_bsr_dev *K, double *work, int cur, hipStream_t s);
const double *cg_scalars(double *work, int64_t n_pad);

}  // namespace pdk
