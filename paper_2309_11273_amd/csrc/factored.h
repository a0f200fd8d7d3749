// Launchers of the factored matrix scheme (factored.hip).
#pragma once

#include "kernels.h"

namespace pdk {

hipError_t launch_fac_assemble(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, hipStream_t s);
hipError_t launch_fac_extension(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, int cur, bool brk,
                                hipStream_t s);
hipError_t launch_fac_kth_dirty(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, int par,
                                hipStream_t s);
hipError_t launch_fac_dilatation(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, hipStream_t s);
hipError_t launch_fac_force(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, int cur, bool update,
                            hipStream_t s);

}  // namespace pdk
