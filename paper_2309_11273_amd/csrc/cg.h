// Launchers of the static solve with the block-sparse stiffness (cg.hip).
#pragma once

#include "kernels.h"

namespace pdk {

int64_t cg_workspace_doubles(int64_t n_pad);
hipError_t launch_cg_start(const StepArgs &a, const pd_bsr_dev *K, double *work, int cur, hipStream_t s);
hipError_t launch_cg_iteration(const StepArgs &a, const pd_bsr_dev *K, double *work, hipStream_t s);
hipError_t launch_cg_finish(const StepArgs &a, const pd_bsr_dev *K, double *work, int cur, hipStream_t s);
const double *cg_scalars(double *work, int64_t n_pad);

}  // namespace pdk
