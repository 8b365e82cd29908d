// Post-synthesis evaluation (Sec. V-A metrics): device view of a hand's
// weighted surface and volume samples, and the launchers of the evaluation
// and top-k kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace grasp {

constexpr int kMaxThresholds = 8;
// Launch shape of the evaluation: a workgroup of kEvalWaves wavefronts takes
// kEvalCandidates candidates and splits their samples between its waves.
#ifndef GRASP_EVAL_CANDIDATES
#define GRASP_EVAL_CANDIDATES 2
#endif
#ifndef GRASP_EVAL_WAVES
#define GRASP_EVAL_WAVES 4
#endif
constexpr int kEvalCandidates = GRASP_EVAL_CANDIDATES;  // one sample load serves them all
constexpr int kEvalWaves = GRASP_EVAL_WAVES;
constexpr int kTopThreads = 1024;
constexpr int kMaxTop = 64;

// Samples of one hand, each set sorted by link: surface samples [0, ns),
// volume samples [ns, ns + nv).
struct EvalView {
  int ns, nv;
  const float4* pts;  // [ns + nv] link-local (x, y, z) and the weight (area or volume)
  const int* link;    // [ns + nv]
};

struct EvalConsts {
  float thr[kMaxThresholds];
  int n_thr;
  float tmax;  // largest threshold: a surface sample provably above it adds nothing
};

// out [B][n_thr + 1]: contact area at each threshold, then the intersection volume.
hipError_t launch_evaluate(const HandView& H, const SdfView& S, const EvalView& E, const EvalConsts& c, int B,
                           const float* q, float* out, hipStream_t stream);

// The same metrics against a mesh object's Phong signed distance; bulge: how
// far the Phong surface can lie from the flat one (alpha times the longest edge).
hipError_t launch_evaluate_mesh(const HandView& H, const MeshView& M, const EvalView& E, const EvalConsts& c,
                                float bulge, int B, const float* q, float* out, hipStream_t stream);

// top [k] (k <= kMaxTop) and mean [M] of metrics [B][M] over them.
hipError_t launch_select_top(int B, const float* key, int higher_is_better, int k, int M, const float* metrics,
                             int* top, float* mean, hipStream_t stream);

}  // namespace grasp
