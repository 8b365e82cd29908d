// Host-side state of a grasp context: device arena, resident hands and SDF
// grids, error reporting. Shared by the C-ABI entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <functional>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "grasp.h"
#include "arena.h"
#include "eval.h"
#include "internal.h"

namespace grasp {

// Thread-local last-error text.
void set_error(const std::string& msg);
grasp_status fail(grasp_status code, const std::string& msg);

struct DevHand {
  HandView view{};
  void* block = nullptr;       // one arena block holding every array
  size_t bytes = 0;
  std::vector<int32_t> contact_link;  // caller order (host copy for validation)
  int live_jobs = 0;
};

struct DevSdf {
  SdfView view{};
  void* block = nullptr;
  size_t bytes = 0;
  float inertia_over_mass = 0.0f;
  int live_jobs = 0;
};

struct DevMesh {
  MeshView view{};
  void* block = nullptr;
  size_t bytes = 0;
  double volume = 0.0;  // enclosed volume (divergence theorem)
  double max_edge = 0.0;  // longest edge: the Phong point is within alpha times it of the flat one
};

struct DevEval {
  EvalView view{};
  void* block = nullptr;
  size_t bytes = 0;
  grasp_hand_id hand = 0;  // the hand whose links the samples hang from
  int live_jobs = 0;       // served jobs that will evaluate with it
};

struct Scheduler;  // serving loop (sched.cpp)

}  // namespace grasp

struct grasp_ctx {
  int device = 0;
  char* arena_base = nullptr;
  bool arena_owned = false;
  grasp::Arena arena;
  std::mutex mu;  // guards the arena and the object tables
  std::map<uint64_t, std::unique_ptr<grasp::DevHand>> hands;
  std::map<uint64_t, std::unique_ptr<grasp::DevSdf>> sdfs;
  std::map<uint64_t, std::unique_ptr<grasp::DevMesh>> meshes;
  std::map<uint64_t, std::unique_ptr<grasp::DevEval>> evals;
  uint64_t next_id = 1;
  std::atomic<bool> poisoned{false};
  std::map<std::string, grasp::TileCfg> tiles;  // tuned launch shapes per problem shape
  grasp::Scheduler* sched = nullptr;  // owned; created and destroyed in sched.cpp
  // candidate locality order of single-job launches: one arena buffer shared
  // by every stream, each use waiting (on the device) for the previous one
  std::mutex order_mu;
  int* order_buf = nullptr;
  int order_cap = 0;
  hipEvent_t order_ev = nullptr;
  // start poses of the Gauss-Seidel sweeps (launches with a backward), shared
  // the same way
  std::mutex gs_mu;
  float* gs_buf = nullptr;
  size_t gs_cap = 0;  // floats
  hipEvent_t gs_ev = nullptr;
  // nearest faces of a one-iteration mesh step's samples (forward to
  // adjoint), shared the same way
  std::mutex face_mu;
  int* face_buf = nullptr;
  size_t face_cap = 0;  // ints
  hipEvent_t face_ev = nullptr;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
};

namespace grasp {

// Makes the context's device current for the scope and restores the
// caller's device afterwards.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
  bool ok() const { return ok_; }

 private:
  int prev_ = -1;
  bool ok_ = false;
};

// HIP failure: poison the context and report EDEVICE.
grasp_status device_fail(grasp_ctx* ctx, hipError_t e, const char* where);

// A usable context: set and not poisoned by an earlier device error.
inline grasp_status check_ctx(grasp_ctx* ctx) {
  if (!ctx) return fail(GRASP_EINVAL, "context is NULL");
  if (ctx->poisoned) return fail(GRASP_EDEVICE, "context poisoned by an earlier device error");
  return GRASP_OK;
}

// Arena sub-allocations inside one block start on 256-byte boundaries.
inline size_t round_up_bytes(size_t x) { return (x + 255) / 256 * 256; }

// Looks up resident objects (caller holds ctx->mu).
DevHand* find_hand(grasp_ctx* ctx, grasp_hand_id id);
DevSdf* find_sdf(grasp_ctx* ctx, grasp_sdf_id id);

// Allocates a grid block (values, block table, gather copy), lets fill write
// the n^3 values at its start (on the device), builds the rest and registers
// the grid. Validation of n, lo, h and the values is the caller's.
grasp_status install_grid(grasp_ctx* ctx, int n, const float lo[3], float h, double Im, int layout,
                          const std::function<hipError_t(float*)>& fill, grasp_sdf_id* out);

// Runs launch(order) with the candidates of q in locality order, or with
// order = null (few candidates, stream capture, no arena room).
hipError_t launch_with_order(grasp_ctx* ctx, const float* q, int n_dof, int B, const SdfView& S, hipStream_t s,
                             const std::function<hipError_t(const int*)>& launch);

// Checks one batch job and resolves its hand, grid and constants.
// gs_ok: the caller also runs Gauss-Seidel jobs (the serving loop does, with
// a launch of their own; the batched launch does not).
grasp_status resolve_job(grasp_ctx* ctx, const grasp_batch_job& j, HandView* h, SdfView* s, StepConsts* c,
                         bool gs_ok = false);

// The serving loop's Gauss-Seidel step: grasp_step_fused without terms or dq,
// its start-pose table at `starts` (gs_scratch_floats(B, n_chunks, K) device
// floats that only stream s uses) instead of the context's shared table;
// *nonfinite (device int) is set when a loss is not finite.
grasp_status step_fused_gs(grasp_ctx* ctx, grasp_hand_id hand, grasp_sdf_id sdf, const grasp_step_params* p,
                           int32_t B, float* q, float* m, float* v, int32_t t, float lr, float b1, float b2, float eps,
                           float* loss, float* starts, int* nonfinite, hipStream_t s);

// Checks step parameters and fills the device constants.
grasp_status check_params(const grasp_step_params* p, StepConsts* out);

}  // namespace grasp
