// Batched form of the grasp step: many jobs (each its own hand, SDF grid,
// candidate count, schedule position) advance one optimizer step in a single
// kernel launch over a device job table. The launch is captured once in a
// hipGraph per launch shape and replayed every step; only the table (copied
// from pinned host memory before each replay) changes between steps.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "batch.h"

using namespace grasp;

namespace grasp {

namespace {

AdamConsts adam_for(int32_t t, float lr, float b1, float b2, float eps) {
  AdamConsts c;
  c.lr = lr;
  c.b1 = b1;
  c.b2 = b2;
  c.eps = eps;
  c.c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(b1), t));
  c.c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(b2), t));
  return c;
}

}  // namespace

// Dilation radius of schedule step t of T (Sec. III-B: linear down to 0).
float dilation_at(float r0, int32_t t, int32_t T) {
  if (T <= 1) return 0.0f;
  const int32_t tt = std::min(t, T - 1);
  return static_cast<float>(static_cast<double>(r0) * (1.0 - static_cast<double>(tt) / (T - 1)));
}

grasp_status batch_fill(grasp_batch* bt, const grasp_batch_job* jobs, int32_t n, int group_kone, int* out_jobs,
                        int* out_total, int* out_lds) {
  // gather the jobs of this kernel group, most expensive candidates first
  std::vector<std::pair<long long, int>> order;
  for (int i = 0; i < n; ++i) {
    const bool kone = jobs[i].p.K == 1;
    if (kone != (group_kone != 0)) continue;
    order.push_back({-static_cast<long long>(bt->views[i].hand.Nc) * jobs[i].p.K, i});
  }
  std::stable_sort(order.begin(), order.end());
  BatchHeader* hdr = reinterpret_cast<BatchHeader*>(bt->host + (group_kone ? 0 : bt->half));
  BatchJob* tab = reinterpret_cast<BatchJob*>(hdr + 1);
  int total = 0, total8 = 0, lds = 0;
  for (size_t k = 0; k < order.size(); ++k) {
    const int i = order[k].second;
    const grasp_batch_job& j = jobs[i];
    BatchJob& e = tab[k];
    std::memset(&e, 0, sizeof(e));
    e.args.hand = bt->views[i].hand;
    e.args.sdf = bt->views[i].sdf;
    e.args.prm = bt->views[i].prm;
    e.args.prm.r_dil = dilation_at(j.r0, j.t, j.T);
    e.args.adam = adam_for(j.t + 1, j.lr, j.b1, j.b2, j.eps);
    e.args.B = j.B;
    e.args.q = j.q;
    e.args.q_out = j.q;
    e.args.m = j.m;
    e.args.v = j.v;
    e.args.loss = j.loss;
    e.args.terms = j.terms;
    e.args.dq = j.dq;
    e.args.nonfinite = bt->flags_dev + i;
    e.args.order = j.B >= kOrderMinB ? bt->order_dev + total : nullptr;
    e.begin = total;
    e.slice = (j.B + 7) / 8;
    e.begin8 = total8;
    total += j.B;
    total8 += e.slice;
    lds = std::max<int>(lds, static_cast<int>(wave_lds_floats(e.args.prm.K, e.args.prm.ckpt)));
  }
  hdr->n_jobs = static_cast<int>(order.size());
  hdr->total = total;
  hdr->total8 = total8;
  *out_jobs = static_cast<int>(order.size());
  *out_total = total;
  *out_lds = lds;
  return GRASP_OK;
}

}  // namespace grasp

extern "C" {

grasp_status grasp_batch_create(grasp_ctx* ctx, int32_t capacity, int32_t max_jobs, int32_t use_graph,
                                grasp_batch** out) {
  set_error("");
  if (!ctx || !out) return fail(GRASP_EINVAL, "ctx/out is NULL");
  if (ctx->poisoned) return fail(GRASP_EDEVICE, "context poisoned");
  if (capacity < 1 || max_jobs < 1 || max_jobs > 4096) return fail(GRASP_EINVAL, "capacity >= 1, 1 <= max_jobs <= 4096");
  auto* bt = new grasp_batch();
  bt->ctx = ctx;
  bt->capacity = capacity;
  bt->max_jobs = max_jobs;
  bt->use_graph = use_graph != 0;
  bt->half = (sizeof(BatchHeader) + static_cast<size_t>(max_jobs) * sizeof(BatchJob) + 255) / 256 * 256;
  // [K=1 table][K>1 table][per-job flags][candidate order, capacity ints]
  const size_t flags_bytes = (static_cast<size_t>(max_jobs) * sizeof(int) + 255) / 256 * 256;
  const size_t bytes = 2 * bt->half + flags_bytes + static_cast<size_t>(capacity) * sizeof(int);
  DeviceGuard g(ctx->device);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    bt->dev = static_cast<char*>(ctx->arena.alloc(bytes));
  }
  if (!bt->dev) {
    delete bt;
    return fail(GRASP_ENOMEM, "arena full (batch table)");
  }
  bt->flags_dev = reinterpret_cast<int*>(bt->dev + 2 * bt->half);
  bt->order_dev = reinterpret_cast<int*>(bt->dev + 2 * bt->half + flags_bytes);
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&bt->host), 2 * bt->half, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemset(bt->flags_dev, 0, static_cast<size_t>(max_jobs) * sizeof(int));
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->arena.free(bt->dev);
    if (bt->host) (void)hipHostFree(bt->host);
    delete bt;
    return device_fail(ctx, e, "grasp_batch_create");
  }
  std::memset(bt->host, 0, 2 * bt->half);
  bt->tile = TileCfg{0, 0};  // unset: each form's default shape
  *out = bt;
  return GRASP_OK;
}

grasp_status grasp_batch_destroy(grasp_batch* bt) {
  set_error("");
  if (!bt) return GRASP_OK;
  DeviceGuard g(bt->ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : bt->graphs) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipGraphDestroy(kv.second.graph);
  }
  if (bt->host) (void)hipHostFree(bt->host);
  {
    std::lock_guard<std::mutex> lk(bt->ctx->mu);
    bt->ctx->arena.free(bt->dev);
  }
  delete bt;
  return GRASP_OK;
}

grasp_status grasp_batch_set_tile(grasp_batch* bt, const grasp_tile* tile) {
  set_error("");
  if (!bt || !tile) return fail(GRASP_EINVAL, "batch/tile is NULL");
  const TileCfg c{tile->waves_per_block, tile->min_waves_per_simd};
  if (!valid_tile(c)) return fail(GRASP_EINVAL, "bad tile");
  bt->tile = c;
  return GRASP_OK;
}

grasp_status grasp_batch_step(grasp_batch* bt, grasp_batch_job* jobs, int32_t n, void* hip_stream) {
  set_error("");
  if (!bt || (n > 0 && !jobs)) return fail(GRASP_EINVAL, "batch/jobs is NULL");
  grasp_ctx* ctx = bt->ctx;
  if (ctx->poisoned) return fail(GRASP_EDEVICE, "context poisoned");
  if (n < 0 || n > bt->max_jobs) return fail(GRASP_EINVAL, "n_jobs out of range");
  bt->views.assign(n, BatchView{});
  long long total = 0;
  for (int i = 0; i < n; ++i) {
    grasp_status st = resolve_job(ctx, jobs[i], &bt->views[i].hand, &bt->views[i].sdf, &bt->views[i].prm);
    if (st != GRASP_OK) return st;
    total += jobs[i].B;
  }
  if (total > bt->capacity) return fail(GRASP_EINVAL, "total candidates exceed the batch capacity");
  if (n == 0) return GRASP_OK;
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  DeviceGuard g(ctx->device);
  hipError_t e = hipSuccess;
  // the table buffers are reused by the next step: wait for the previous one
  if (bt->last) e = hipEventSynchronize(bt->last);
  for (int group = 1; group >= 0 && e == hipSuccess; --group) {
    int nj = 0, tot = 0, lds = 0;
    batch_fill(bt, jobs, n, group, &nj, &tot, &lds);
    if (nj == 0) continue;
    const size_t off = group ? 0 : bt->half;
    const size_t bytes = sizeof(BatchHeader) + static_cast<size_t>(nj) * sizeof(BatchJob);
    e = hipMemcpyAsync(bt->dev + off, bt->host + off, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) break;
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(bt->dev + off);
    const BatchJob* tab = reinterpret_cast<const BatchJob*>(hdr + 1);
    const TileCfg tc = valid_tile(bt->tile) ? bt->tile : default_tile(group != 0);
    bool fric = false;  // a job of this group with friction
    for (int i = 0; i < n; ++i)
      if ((bt->views[i].prm.K == 1) == (group != 0) && bt->views[i].prm.mu > 0.0f) fric = true;
    // every XCD's list holds at most capacity / 8 + max_jobs candidates
    const int per_xcd = (bt->capacity + 7) / 8 + bt->max_jobs;
    const int blocks = 8 * ((per_xcd + tc.wpb - 1) / tc.wpb);
    if (!bt->use_graph || s == nullptr) {
      e = launch_order_batch(hdr, tab, bt->max_jobs, s);
      if (e == hipSuccess) e = launch_batch(hdr, tab, group != 0, fric, tc, blocks, lds, s);
      continue;
    }
    const auto key = std::make_tuple(group + (fric ? 2 : 0), tc.wpb, tc.occ, lds);
    auto it = bt->graphs.find(key);
    if (it == bt->graphs.end()) {
      BatchGraph bg{};
      e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
      if (e == hipSuccess) {
        hipError_t le = launch_order_batch(hdr, tab, bt->max_jobs, s);
        if (le == hipSuccess) le = launch_batch(hdr, tab, group != 0, fric, tc, blocks, lds, s);
        e = hipStreamEndCapture(s, &bg.graph);
        if (e == hipSuccess) e = le;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&bg.exec, bg.graph, nullptr, nullptr, 0);
      if (e != hipSuccess) break;
      it = bt->graphs.emplace(key, bg).first;
    }
    e = hipGraphLaunch(it->second.exec, s);
  }
  if (e == hipSuccess && !bt->last) e = hipEventCreateWithFlags(&bt->last, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(bt->last, s);
  if (e != hipSuccess) return device_fail(ctx, e, "grasp_batch_step");
  for (int i = 0; i < n; ++i) jobs[i].t += 1;
  return GRASP_OK;
}

grasp_status grasp_batch_flags(grasp_batch* bt, int32_t n, int32_t* out) {
  set_error("");
  if (!bt || !out || n < 0 || n > bt->max_jobs) return fail(GRASP_EINVAL, "bad arguments");
  DeviceGuard g(bt->ctx->device);
  // the flags are written by the last step, which may run on any stream
  hipError_t e = bt->last ? hipEventSynchronize(bt->last) : hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(out, bt->flags_dev, static_cast<size_t>(n) * sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(bt->flags_dev, 0, static_cast<size_t>(n) * sizeof(int));
  if (e != hipSuccess) return device_fail(bt->ctx, e, "grasp_batch_flags");
  return GRASP_OK;
}

}  // extern "C"
