// Launchers of the finite-deformation force kernels (finite.hip).
#pragma once

#include "kernels.h"

namespace pdk {

hipError_t launch_fin_pass1(const StepArgs &a, int cur, bool brk, int block, hipStream_t s);
hipError_t launch_fin_pass2(const StepArgs &a, int cur, bool update, int block, hipStream_t s);
// the finite model in the LDS-staged double-precision tile kernels
bool tiled64_fin_supported(const StepArgs &a);
hipError_t launch_tpass1_f64_fin(const StepArgs &a, int cur, bool brk, hipStream_t s);
hipError_t launch_tpass2_f64_fin(const StepArgs &a, int cur, bool update, hipStream_t s);

}  // namespace pdk
