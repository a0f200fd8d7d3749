// Launchers of the adaptive dynamic relaxation (adr.hip).
#pragma once

#include "kernels.h"

namespace pdk {

int adr_blocks(int64_t n_pad);
hipError_t launch_adr_density(const StepArgs &a, const pd_problem_dev *p, const pd_adr_dev *R, hipStream_t s);
hipError_t launch_adr_iteration(const StepArgs &a, const pd_problem_dev *p, const pd_adr_dev *R, int cur,
                                hipStream_t s);

}  // namespace pdk
