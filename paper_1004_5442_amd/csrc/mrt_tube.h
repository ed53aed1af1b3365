// mrt_tube.h -- constants of the tube march shared by its kernel
// (tube_kernel, mrt_kernels.hip) and the host library (mrt_api.hip).
#pragma once

namespace mrt {

// Time steps per pass, and the columns one block stores: its 256 lanes less
// the recomputed overlap of one column per step on either side.
constexpr int kTubeSteps = 4;
constexpr int kTubeWidth = 256 - 2 * kTubeSteps;

}  // namespace mrt
