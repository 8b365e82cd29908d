// Serving on the device: the executor of the serving loop (serve_core.h) for
// a grasp context, and the C entry points grasp_serve_config, grasp_submit,
// grasp_poll, grasp_cancel and grasp_serve_stats_get.
//
// A resident job holds one arena block: q, m, v, loss, terms; with an
// evaluation set its metrics, top-k indices and mean metrics; a
// Gauss-Seidel job also its sweep start-pose table and a non-finite flag.
// Every resident averaged job advances by one batched launch per step
// (grasp_batch_step, graph-replayed on the executor's stream); a
// Gauss-Seidel job by a fused launch of its own on the same stream. Every
// candidate is computed by the same per-candidate code as the single-job
// step, so a job's results do not depend on which other jobs shared its
// steps. Retiring a job runs one forward at r_dil = 0 (final loss and terms),
// the optional evaluation and top-k, and copies the results to the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <vector>

#include "batch.h"
#include "gs.h"
#include "serve_core.h"

using namespace grasp;

namespace grasp {

namespace {

size_t r256(size_t x) { return (x + 255) / 256 * 256; }

int job_metrics(const grasp_job_desc& d) { return d.eval ? d.n_thr + 1 : 0; }

// Byte offsets of a job's arrays inside its arena block.
struct JobLayout {
  size_t q, m, v, loss, terms, metrics, top, mean, starts, flag, total;
};

JobLayout job_layout(int B, int n_dof, int M, int top_k, size_t start_floats) {
  const size_t b = static_cast<size_t>(B);
  JobLayout L{};
  const size_t nq = r256(b * n_dof * 4);
  L.q = 0;
  L.m = nq;
  L.v = 2 * nq;
  L.loss = 3 * nq;
  L.terms = L.loss + r256(b * 4);
  size_t o = L.terms + r256(b * 16);
  if (M > 0) {
    L.metrics = o;
    L.top = o + r256(b * M * 4);
    L.mean = L.top + r256(static_cast<size_t>(top_k) * 4);
    o = L.mean + r256(static_cast<size_t>(M) * 4);
  }
  if (start_floats) {
    L.starts = o;
    L.flag = o + r256(start_floats * 4);
    o = L.flag + 256;
  }
  L.total = o;
  return L;
}

struct DevJob {
  void* block = nullptr;
  float *q = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr, *terms = nullptr;
  float *metrics = nullptr, *mean = nullptr, *starts = nullptr;
  int32_t* top = nullptr;
  int* flag = nullptr;
  size_t start_floats = 0;
};

DevJob* dev_of(ServeJob& j) { return static_cast<DevJob*>(j.exec); }

class DeviceExecutor final : public ServeExecutor {
 public:
  explicit DeviceExecutor(grasp_ctx* ctx) : ctx_(ctx) {}
  ~DeviceExecutor() override {
    DeviceGuard g(ctx_->device);
    if (batch_) grasp_batch_destroy(batch_);
    if (stream_) (void)hipStreamDestroy(stream_);
  }
  grasp_status open(int32_t capacity, int32_t max_jobs) {
    DeviceGuard g(ctx_->device);
    hipError_t e = hipStreamCreate(&stream_);
    if (e != hipSuccess) return device_fail(ctx_, e, "scheduler stream");
    return grasp_batch_create(ctx_, capacity, max_jobs, 1, &batch_);
  }

  grasp_status admit(ServeJob& j) override {
    DevJob* d = dev_of(j);
    void* blk = nullptr;
    {
      std::lock_guard<std::mutex> lk(ctx_->mu);
      blk = ctx_->arena.alloc(j.footprint);
    }
    if (!blk) return GRASP_EAGAIN;
    const JobLayout L = job_layout(j.desc.B, j.n_dof, job_metrics(j.desc), j.desc.eval ? j.desc.top_k : 0,
                                   d->start_floats);
    char* p = static_cast<char*>(blk);
    d->block = blk;
    d->q = reinterpret_cast<float*>(p + L.q);
    d->m = reinterpret_cast<float*>(p + L.m);
    d->v = reinterpret_cast<float*>(p + L.v);
    d->loss = reinterpret_cast<float*>(p + L.loss);
    d->terms = reinterpret_cast<float*>(p + L.terms);
    if (job_metrics(j.desc) > 0) {
      d->metrics = reinterpret_cast<float*>(p + L.metrics);
      d->top = reinterpret_cast<int32_t*>(p + L.top);
      d->mean = reinterpret_cast<float*>(p + L.mean);
    }
    if (d->start_floats) {
      d->starts = reinterpret_cast<float*>(p + L.starts);
      d->flag = reinterpret_cast<int*>(p + L.flag);
    }
    const size_t nq = static_cast<size_t>(j.desc.B) * j.n_dof * 4;
    DeviceGuard g(ctx_->device);
    hipError_t e = hipMemcpyAsync(d->q, j.q0.data(), nq, hipMemcpyHostToDevice, stream_);
    if (e == hipSuccess) e = hipMemsetAsync(d->m, 0, L.loss - L.m, stream_);
    if (e == hipSuccess && d->flag) e = hipMemsetAsync(d->flag, 0, sizeof(int), stream_);
    if (e == hipSuccess) e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) return device_fail(ctx_, e, "scheduler admission");
    if (j.desc.record_history) {
      j.hist_q.assign(static_cast<size_t>(j.desc.T) * j.desc.B * j.n_dof, 0.0f);
      j.hist_loss.assign(static_cast<size_t>(j.desc.T) * j.desc.B, 0.0f);
    }
    return GRASP_OK;
  }

  grasp_status step(const std::vector<ServeJob*>& jobs, std::vector<grasp_status>& st) override {
    DeviceGuard g(ctx_->device);
    bj_.clear();
    bjob_.clear();
    gsjob_.clear();
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < jobs.size(); ++k) {
      ServeJob& j = *jobs[k];
      DevJob* d = dev_of(j);
      if (j.desc.record_history && e == hipSuccess)
        e = hipMemcpyAsync(j.hist_q.data() + static_cast<size_t>(j.t) * j.desc.B * j.n_dof, d->q,
                           static_cast<size_t>(j.desc.B) * j.n_dof * 4, hipMemcpyDeviceToHost, stream_);
      if (j.desc.p.projection == GRASP_PROJECTION_GAUSS_SEIDEL) {
        gsjob_.push_back(k);  // stepped by a launch of its own
        continue;
      }
      grasp_batch_job b{};
      b.hand = j.desc.hand;
      b.sdf = j.desc.sdf;
      b.p = j.desc.p;
      b.B = j.desc.B;
      b.q = d->q;
      b.m = d->m;
      b.v = d->v;
      b.loss = d->loss;
      b.t = j.t;
      b.T = j.desc.T;
      b.r0 = j.desc.r0;
      b.lr = j.desc.lr;
      b.b1 = j.desc.b1;
      b.b2 = j.desc.b2;
      b.eps = j.desc.eps;
      bj_.push_back(b);
      bjob_.push_back(k);
    }
    if (e != hipSuccess) return device_fail(ctx_, e, "scheduler history");
    flags_.assign(bj_.size(), 0);
    if (!bj_.empty()) {
      grasp_status s = grasp_batch_step(batch_, bj_.data(), static_cast<int32_t>(bj_.size()), stream_);
      if (s == GRASP_OK) s = grasp_batch_flags(batch_, static_cast<int32_t>(bj_.size()), flags_.data());
      if (s != GRASP_OK) return s;
    }
    for (size_t i = 0; i < bjob_.size(); ++i)
      if (flags_[i]) st[bjob_[i]] = GRASP_ENONFINITE;
    // Gauss-Seidel jobs: the same dilation schedule, their own start-pose table
    for (size_t k : gsjob_) {
      ServeJob& j = *jobs[k];
      DevJob* d = dev_of(j);
      grasp_step_params p = j.desc.p;
      p.r_dil = dilation_at(j.desc.r0, j.t, j.desc.T);
      const grasp_status s = step_fused_gs(ctx_, j.desc.hand, j.desc.sdf, &p, j.desc.B, d->q, d->m, d->v, j.t + 1,
                                           j.desc.lr, j.desc.b1, j.desc.b2, j.desc.eps, d->loss, d->starts, d->flag,
                                           stream_);
      if (s == GRASP_EDEVICE) return s;
      st[k] = s;  // a refusal ends this job only
    }
    std::vector<int> gflag(gsjob_.size(), 0);
    for (size_t i = 0; i < gsjob_.size() && e == hipSuccess; ++i) {
      DevJob* d = dev_of(*jobs[gsjob_[i]]);
      if (st[gsjob_[i]] != GRASP_OK) continue;
      e = hipMemcpyAsync(&gflag[i], d->flag, sizeof(int), hipMemcpyDeviceToHost, stream_);
      if (e == hipSuccess) e = hipMemsetAsync(d->flag, 0, sizeof(int), stream_);
    }
    for (size_t k = 0; k < jobs.size() && e == hipSuccess; ++k) {
      ServeJob& j = *jobs[k];
      if (j.desc.record_history)
        e = hipMemcpyAsync(j.hist_loss.data() + static_cast<size_t>(j.t) * j.desc.B, dev_of(j)->loss,
                           static_cast<size_t>(j.desc.B) * 4, hipMemcpyDeviceToHost, stream_);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) return device_fail(ctx_, e, "scheduler step");
    for (size_t i = 0; i < gsjob_.size(); ++i)
      if (gflag[i]) st[gsjob_[i]] = GRASP_ENONFINITE;
    return GRASP_OK;
  }

  void finish(ServeJob& j) override {
    DevJob* d = dev_of(j);
    const int B = j.desc.B;
    DeviceGuard g(ctx_->device);
    if (j.status == GRASP_OK) {
      grasp_step_params p = j.desc.p;
      p.r_dil = 0.0f;
      p.mode = GRASP_MODE_RECOMPUTE;
      grasp_status st = grasp_step_fwd(ctx_, j.desc.hand, j.desc.sdf, &p, B, d->q, d->loss, d->terms, nullptr, 0,
                                       stream_);
      // post-synthesis evaluation at the final configurations, then the best by final loss
      if (st == GRASP_OK && d->metrics)
        st = grasp_evaluate(ctx_, j.desc.eval, j.desc.sdf, B, d->q, j.desc.n_thr, j.desc.thresholds, d->metrics,
                            stream_);
      if (st == GRASP_OK && d->metrics && j.desc.top_k > 0)
        st = grasp_select_top(ctx_, B, d->loss, 0, j.desc.top_k, j.desc.n_thr + 1, d->metrics, d->top, d->mean,
                              stream_);
      if (st != GRASP_OK) j.status = st;
    }
    j.out_q.resize(static_cast<size_t>(B) * j.n_dof);
    j.out_loss.resize(B);
    j.out_terms.resize(static_cast<size_t>(B) * 4);
    hipError_t e = hipStreamSynchronize(stream_);
    if (e == hipSuccess) e = hipMemcpy(j.out_q.data(), d->q, j.out_q.size() * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(j.out_loss.data(), d->loss, j.out_loss.size() * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(j.out_terms.data(), d->terms, j.out_terms.size() * 4, hipMemcpyDeviceToHost);
    if (d->metrics && j.status == GRASP_OK) {
      const size_t M = static_cast<size_t>(j.desc.n_thr) + 1;
      j.out_metrics.resize(static_cast<size_t>(B) * M);
      if (e == hipSuccess)
        e = hipMemcpy(j.out_metrics.data(), d->metrics, j.out_metrics.size() * 4, hipMemcpyDeviceToHost);
      if (j.desc.top_k > 0) {
        j.out_top.resize(j.desc.top_k);
        j.out_mean.resize(M);
        if (e == hipSuccess) e = hipMemcpy(j.out_top.data(), d->top, j.out_top.size() * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(j.out_mean.data(), d->mean, M * 4, hipMemcpyDeviceToHost);
      }
    }
    if (e != hipSuccess) {
      j.status = device_fail(ctx_, e, "scheduler results");
      throw std::runtime_error("device failure");
    }
    if (j.status == GRASP_OK)
      for (float x : j.out_loss)
        if (!std::isfinite(x)) j.status = GRASP_ENONFINITE;
    j.rank = rank_by_loss(j.out_loss);
  }

  void drain() override {
    DeviceGuard g(ctx_->device);
    const hipError_t e = hipStreamSynchronize(stream_);
    if (e != hipSuccess) {
      (void)device_fail(ctx_, e, "scheduler drain");
      throw std::runtime_error("device failure");
    }
  }

  void release(ServeJob& j) override {
    std::unique_ptr<DevJob> d(dev_of(j));
    j.exec = nullptr;
    std::lock_guard<std::mutex> lk(ctx_->mu);
    if (d && d->block) ctx_->arena.free(d->block);
    if (DevHand* h = find_hand(ctx_, j.desc.hand)) h->live_jobs--;
    if (DevSdf* s = find_sdf(ctx_, j.desc.sdf)) s->live_jobs--;
    if (j.desc.eval) {
      auto it = ctx_->evals.find(j.desc.eval);
      if (it != ctx_->evals.end()) it->second->live_jobs--;
    }
  }

 private:
  grasp_ctx* ctx_;
  grasp_batch* batch_ = nullptr;
  hipStream_t stream_ = nullptr;
  std::vector<grasp_batch_job> bj_;
  std::vector<size_t> bjob_, gsjob_;
  std::vector<int32_t> flags_;
};

}  // namespace

struct Scheduler {
  std::unique_ptr<DeviceExecutor> exec;
  std::unique_ptr<ServeLoop> loop;
  int32_t capacity = 65536, max_jobs = 256;
  std::mutex open_mu;
  bool opened = false;
};

}  // namespace grasp

namespace {

Scheduler* sched_of(grasp_ctx* ctx) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->sched) {
    auto* s = new Scheduler();
    s->exec = std::make_unique<DeviceExecutor>(ctx);
    s->loop = std::make_unique<ServeLoop>(s->exec.get(), [ctx] {
      return std::chrono::duration<double>(std::chrono::steady_clock::now() - ctx->t0).count();
    });
    ctx->sched = s;
  }
  return ctx->sched;
}

grasp_status status_error(grasp_status st, const char* what) {
  return st == GRASP_OK || st == GRASP_EAGAIN ? st : fail(st, what);
}

}  // namespace

extern "C" {

void grasp_shutdown_scheduler(grasp_ctx* ctx) {
  if (!ctx || !ctx->sched) return;
  Scheduler* s = ctx->sched;
  s->loop->shutdown();
  s->loop.reset();
  s->exec.reset();
  delete s;
  ctx->sched = nullptr;
}

grasp_status grasp_serve_config(grasp_ctx* ctx, int32_t capacity, int32_t max_jobs) {
  set_error("");
  if (!ctx) return fail(GRASP_EINVAL, "context is NULL");
  Scheduler* s = sched_of(ctx);
  const grasp_status st = s->loop->configure(capacity, max_jobs);
  if (st == GRASP_EINVAL) return fail(st, "bad capacity / max_jobs");
  if (st == GRASP_EBUSY) return fail(st, "the scheduler is already running");
  s->capacity = capacity;
  s->max_jobs = max_jobs;
  return GRASP_OK;
}

grasp_status grasp_submit(grasp_ctx* ctx, const grasp_job_desc* d, grasp_job_id* out) {
  set_error("");
  if (!ctx || !d || !out) return fail(GRASP_EINVAL, "ctx/job/out is NULL");
  if (ctx->poisoned) return fail(GRASP_EDEVICE, "context poisoned");
  if (d->B < 1 || !d->q0 || d->T < 1 || !(d->r0 >= 0.0f))
    return fail(GRASP_EINVAL, "job needs B >= 1, q0, T >= 1, r0 >= 0");
  if (d->record_history != 0 && d->record_history != 1) return fail(GRASP_EINVAL, "record_history must be 0 or 1");
  int n_dof = 0, nc = 0;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    DevHand* h = find_hand(ctx, d->hand);
    DevSdf* s = find_sdf(ctx, d->sdf);
    if (!h || !s) return fail(GRASP_EINVAL, "unknown hand or sdf id");
    n_dof = h->view.n_dof;
    nc = h->view.Nc;
  }
  grasp_batch_job probe{};
  probe.hand = d->hand;
  probe.sdf = d->sdf;
  probe.p = d->p;
  probe.B = d->B;
  probe.q = probe.m = probe.v = reinterpret_cast<float*>(16);  // only checked for presence
  probe.T = d->T;
  probe.r0 = d->r0;
  probe.lr = d->lr;
  probe.b1 = d->b1;
  probe.b2 = d->b2;
  probe.eps = d->eps;
  HandView hv;
  SdfView sv;
  StepConsts sc;
  grasp_status st = resolve_job(ctx, probe, &hv, &sv, &sc, true);
  if (st != GRASP_OK) return st;
  if (d->eval) {
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      auto it = ctx->evals.find(d->eval);
      if (it == ctx->evals.end()) return fail(GRASP_EINVAL, "unknown evaluation set id");
      if (it->second->hand != d->hand) return fail(GRASP_EINVAL, "the evaluation set belongs to another hand");
    }
    if (d->n_thr < 1 || d->n_thr > GRASP_MAX_THRESHOLDS) return fail(GRASP_EINVAL, "n_thr must be in [1, 8]");
    for (int t = 0; t < d->n_thr; ++t)
      if (!std::isfinite(d->thresholds[t])) return fail(GRASP_EINVAL, "thresholds must be finite");
    if (d->top_k < 0 || d->top_k > std::min(d->B, GRASP_MAX_TOP))
      return fail(GRASP_EINVAL, "top_k must be in [0, min(B, 64)]");
  } else if (d->top_k != 0) {
    return fail(GRASP_EINVAL, "top_k needs an evaluation set");
  }
  Scheduler* s = sched_of(ctx);
  {
    // the executor's stream and batch exist from the first submission on
    std::lock_guard<std::mutex> lk(s->open_mu);
    if (!s->opened) {
      st = s->exec->open(s->capacity, s->max_jobs);
      if (st != GRASP_OK) return st;
      s->opened = true;
    }
  }
  auto j = std::make_unique<ServeJob>();
  j->desc = *d;
  j->n_dof = n_dof;
  j->n_contacts = nc;
  auto dj = std::make_unique<DevJob>();
  // a Gauss-Seidel job keeps its own start-pose table, reserved at admission
  dj->start_floats =
      d->p.projection == GRASP_PROJECTION_GAUSS_SEIDEL ? gs_scratch_floats(d->B, hv.n_chunks, d->p.K) : 0;
  j->footprint =
      job_layout(d->B, n_dof, job_metrics(*d), d->eval ? d->top_k : 0, dj->start_floats).total;
  j->q0.assign(d->q0, d->q0 + static_cast<size_t>(d->B) * n_dof);
  j->desc.q0 = nullptr;
  DevJob* dev_state = dj.release();
  j->exec = dev_state;
  // the job's references to its hand, grid and evaluation set, taken when it is queued
  auto take_refs = [ctx, d] {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (DevHand* h = find_hand(ctx, d->hand)) h->live_jobs++;
    if (DevSdf* g = find_sdf(ctx, d->sdf)) g->live_jobs++;
    if (d->eval) {
      auto it = ctx->evals.find(d->eval);
      if (it != ctx->evals.end()) it->second->live_jobs++;
    }
  };
  st = s->loop->submit(std::move(j), ctx->arena.capacity(), take_refs, out);
  if (st != GRASP_OK) {
    delete dev_state;  // the loop did not take the job
    if (st == GRASP_ENOMEM) return fail(st, "job can never fit the candidate capacity or the arena");
    if (st == GRASP_EDEVICE) return fail(st, "the serving loop stopped after a device error");
    return fail(st, "the serving loop is shutting down");
  }
  return GRASP_OK;
}

grasp_status grasp_poll(grasp_ctx* ctx, grasp_job_id id, grasp_job_result* r) {
  set_error("");
  if (!ctx || !r) return fail(GRASP_EINVAL, "ctx/result is NULL");
  if (!ctx->sched) return fail(GRASP_EINVAL, "unknown job id");
  const grasp_status st = ctx->sched->loop->poll(id, r);
  if (st == GRASP_EINVAL) return fail(st, "unknown job id");
  return status_error(st, "job ended with a non-OK status");
}

grasp_status grasp_cancel(grasp_ctx* ctx, grasp_job_id id) {
  set_error("");
  if (!ctx || !ctx->sched) return fail(GRASP_EINVAL, "unknown job id");
  const grasp_status st = ctx->sched->loop->cancel(id);
  return st == GRASP_OK ? st : fail(st, "unknown job id");
}

grasp_status grasp_serve_stats_get(grasp_ctx* ctx, grasp_serve_stats* out) {
  set_error("");
  if (!ctx || !out) return fail(GRASP_EINVAL, "ctx/out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!ctx->sched) return GRASP_OK;
  ctx->sched->loop->stats(out);
  return GRASP_OK;
}

}  // extern "C"
