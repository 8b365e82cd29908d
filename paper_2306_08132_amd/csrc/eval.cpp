// Post-synthesis evaluation (Sec. V-A metrics), host side: the hand's
// weighted surface and volume samples and the C-ABI entry points of the
// evaluation and top-k kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "grasp.h"
#include "context.h"
#include "eval.h"

using namespace grasp;

namespace {

// One sample set checked and appended in link order (stable within a link).
grasp_status append_set(int n, const int32_t* link, const float* local, const float* w, int L, const char* what,
                        std::vector<float4>& pts, std::vector<int>& links) {
  if (n < 0 || n > (1 << 24)) return fail(GRASP_EINVAL, std::string(what) + " count must be in [0, 2^24]");
  if (n == 0) return GRASP_OK;
  if (!link || !local || !w) return fail(GRASP_EINVAL, std::string(what) + " arrays are NULL");
  for (int i = 0; i < n; ++i) {
    if (link[i] < 0 || link[i] >= L) return fail(GRASP_EINVAL, std::string(what) + " link out of range");
    if (!std::isfinite(local[3 * i]) || !std::isfinite(local[3 * i + 1]) || !std::isfinite(local[3 * i + 2]))
      return fail(GRASP_EINVAL, std::string(what) + " coordinates must be finite");
    if (!std::isfinite(w[i]) || w[i] < 0.0f) return fail(GRASP_EINVAL, std::string(what) + " weights must be finite and >= 0");
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return link[a] < link[b]; });
  for (int i : order) {
    pts.push_back(make_float4(local[3 * i], local[3 * i + 1], local[3 * i + 2], w[i]));
    links.push_back(link[i]);
  }
  return GRASP_OK;
}

}  // namespace

extern "C" {

grasp_status grasp_load_eval_points(grasp_ctx* ctx, grasp_hand_id hand, const grasp_eval_desc* d,
                                    grasp_eval_id* out) {
  set_error("");
  if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
  if (!d || !out) return fail(GRASP_EINVAL, "desc/out is NULL");
  int L;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    DevHand* h = find_hand(ctx, hand);
    if (!h) return fail(GRASP_EINVAL, "unknown hand id");
    L = h->view.L;
  }
  std::vector<float4> pts;
  std::vector<int> links;
  grasp_status st = append_set(d->n_surface, d->surface_link, d->surface_local, d->surface_area, L, "surface sample",
                               pts, links);
  if (st != GRASP_OK) return st;
  st = append_set(d->n_volume, d->volume_link, d->volume_local, d->volume_weight, L, "volume sample", pts, links);
  if (st != GRASP_OK) return st;
  if (pts.empty()) return fail(GRASP_EINVAL, "no samples");
  const size_t bp = round_up_bytes(pts.size() * sizeof(float4)), bl = round_up_bytes(links.size() * sizeof(int));
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(GRASP_EDEVICE, "hipSetDevice failed");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!find_hand(ctx, hand)) return fail(GRASP_EINVAL, "unknown hand id");
  void* blk = ctx->arena.alloc(bp + bl);
  if (!blk) return fail(GRASP_ENOMEM, "arena full (evaluation samples)");
  char* b = static_cast<char*>(blk);
  hipError_t e = hipMemcpy(b, pts.data(), pts.size() * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b + bp, links.data(), links.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    ctx->arena.free(blk);
    return device_fail(ctx, e, "evaluation sample upload");
  }
  auto ev = std::make_unique<DevEval>();
  ev->view.ns = d->n_surface;
  ev->view.nv = d->n_volume;
  ev->view.pts = reinterpret_cast<const float4*>(b);
  ev->view.link = reinterpret_cast<const int*>(b + bp);
  ev->block = blk;
  ev->bytes = bp + bl;
  ev->hand = hand;
  const uint64_t id = ctx->next_id++;
  ctx->evals[id] = std::move(ev);
  *out = id;
  return GRASP_OK;
}

grasp_status grasp_unload_eval_points(grasp_ctx* ctx, grasp_eval_id id) {
  set_error("");
  if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->evals.find(id);
  if (it == ctx->evals.end()) return fail(GRASP_EINVAL, "unknown evaluation set id");
  if (it->second->live_jobs > 0) return fail(GRASP_EBUSY, "evaluation set in use by a live job");
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->arena.free(it->second->block);
  ctx->evals.erase(it);
  return GRASP_OK;
}

}  // extern "C"

namespace {

// Checks the call and the thresholds; resolves the set and its hand.
grasp_status eval_args(grasp_ctx* ctx, grasp_eval_id id, int32_t B, const float* q, int32_t n_thr,
                       const float* thresholds, float* out, EvalConsts* c, HandView* hv, EvalView* ev) {
  if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
  if (B < 0 || B > (1 << 26)) return fail(GRASP_EINVAL, "B must be in [0, 2^26]");
  if (n_thr < 1 || n_thr > kMaxThresholds) return fail(GRASP_EINVAL, "n_thr must be in [1, 8]");
  if (!thresholds) return fail(GRASP_EINVAL, "thresholds is NULL");
  if (B > 0 && (!q || !out)) return fail(GRASP_EINVAL, "q/out is NULL");
  *c = EvalConsts{};
  c->n_thr = n_thr;
  c->tmax = -INFINITY;
  for (int t = 0; t < n_thr; ++t) {
    if (!std::isfinite(thresholds[t])) return fail(GRASP_EINVAL, "thresholds must be finite");
    c->thr[t] = thresholds[t];
    c->tmax = std::max(c->tmax, thresholds[t]);
  }
  auto it = ctx->evals.find(id);
  if (it == ctx->evals.end()) return fail(GRASP_EINVAL, "unknown evaluation set id");
  DevHand* h = find_hand(ctx, it->second->hand);
  if (!h) return fail(GRASP_EINVAL, "the evaluation set's hand no longer exists");
  *hv = h->view;
  *ev = it->second->view;
  return GRASP_OK;
}

}  // namespace

extern "C" {

grasp_status grasp_evaluate(grasp_ctx* ctx, grasp_eval_id id, grasp_sdf_id sdf, int32_t B, const float* q,
                            int32_t n_thr, const float* thresholds, float* out, void* hip_stream) {
  set_error("");
  EvalConsts c;
  HandView hv;
  SdfView sv;
  EvalView ev;
  {
    if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (const grasp_status st = eval_args(ctx, id, B, q, n_thr, thresholds, out, &c, &hv, &ev); st != GRASP_OK)
      return st;
    DevSdf* s = find_sdf(ctx, sdf);
    if (!s) return fail(GRASP_EINVAL, "unknown sdf id");
    sv = s->view;
  }
  DeviceGuard g(ctx->device);
  const hipError_t e = launch_evaluate(hv, sv, ev, c, B, q, out, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_evaluate launch");
  return GRASP_OK;
}

grasp_status grasp_evaluate_mesh(grasp_ctx* ctx, grasp_eval_id id, grasp_mesh_id mesh, int32_t B, const float* q,
                                 int32_t n_thr, const float* thresholds, float* out, void* hip_stream) {
  set_error("");
  EvalConsts c;
  HandView hv;
  MeshView mv;
  EvalView ev;
  float bulge;
  {
    if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (const grasp_status st = eval_args(ctx, id, B, q, n_thr, thresholds, out, &c, &hv, &ev); st != GRASP_OK)
      return st;
    auto it = ctx->meshes.find(mesh);
    if (it == ctx->meshes.end()) return fail(GRASP_EINVAL, "unknown mesh id");
    mv = it->second->view;
    bulge = static_cast<float>(mv.alpha * it->second->max_edge * (1.0 + 1e-6));
  }
  DeviceGuard g(ctx->device);
  const hipError_t e = launch_evaluate_mesh(hv, mv, ev, c, bulge, B, q, out, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_evaluate_mesh launch");
  return GRASP_OK;
}

grasp_status grasp_select_top(grasp_ctx* ctx, int32_t B, const float* key, int32_t higher_is_better, int32_t k,
                              int32_t M, const float* metrics, int32_t* top, float* mean, void* hip_stream) {
  set_error("");
  if (const grasp_status st = check_ctx(ctx); st != GRASP_OK) return st;
  if (B < 1 || B > (1 << 24)) return fail(GRASP_EINVAL, "B must be in [1, 2^24]");
  if (k < 1 || k > std::min(B, kMaxTop)) return fail(GRASP_EINVAL, "k must be in [1, min(B, 64)]");
  if (M < 0 || M > (1 << 16)) return fail(GRASP_EINVAL, "M must be in [0, 2^16]");
  if (!key || !top) return fail(GRASP_EINVAL, "key/top is NULL");
  if (M > 0 && (!metrics || !mean)) return fail(GRASP_EINVAL, "metrics/mean is NULL");
  DeviceGuard g(ctx->device);
  const hipError_t e = launch_select_top(B, key, higher_is_better, k, M, metrics, top, mean,
                                         static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_select_top launch");
  return GRASP_OK;
}

}  // extern "C"
