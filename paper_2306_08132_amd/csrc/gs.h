// Gauss-Seidel projection of the grasp step (Sec. III-C): launcher of the
// wave-serial sweep kernel and its LDS footprint.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace grasp {

constexpr int kGsWaves = 2;             // candidates (waves) per workgroup

// Floats of the start-pose table a launch with a backward needs: the pose of
// every (candidate, iteration, 64-contact chunk, test) where a chunk's sweep
// begins.
size_t gs_scratch_floats(int B, int n_chunks, int K);

// One step with the constraints swept one after another: loss and
// terms (kind != STEP_BWD), dq and Adam as the averaged step's launch.
// starts: the start-pose table (device, gs_scratch_floats) unless kind is
// STEP_FWD, where it may be null.
hipError_t launch_gs_step(const StepArgs& a, StepKind kind, bool adam, float* starts, hipStream_t stream);

}  // namespace grasp
