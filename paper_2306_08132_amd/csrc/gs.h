// Gauss-Seidel projection of the grasp step (Sec. III-C): launcher of the
// wave-serial sweep kernel and its LDS footprint.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace grasp {

constexpr int kGsWaves = 2;             // candidates (waves) per workgroup
constexpr int kGsMaxContacts = 8192;    // chunk start poses of every test stay in LDS

// LDS floats of one wave for a hand of n_chunks 64-contact chunks.
size_t gs_lds_floats(int n_chunks);

// One step with K = 1 and the constraints swept one after another: loss and
// terms (kind != STEP_BWD), dq and Adam as the averaged step's launch.
hipError_t launch_gs_step(const StepArgs& a, StepKind kind, bool adam, hipStream_t stream);

}  // namespace grasp
