// Launchers of the finite-deformation force kernels (finite.hip).
#pragma once

#include "kernels.h"

namespace pdk {

hipError_t launch_fin_pass1(const StepArgs &a, int cur, bool brk, int block, hipStream_t s);
hipError_t launch_fin_pass2(const StepArgs &a, int cur, bool update, int block, hipStream_t s);

}  // namespace pdk
