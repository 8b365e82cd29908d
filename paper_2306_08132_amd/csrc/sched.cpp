// Serving loop of the grasp library: continuous batching of grasp jobs.
//
// grasp_submit copies a job into the queue. A scheduler thread (one per
// context, started by the first submit) repeats, at every step boundary:
//   1. end cancelled jobs;
//   2. admit queued jobs in arrival order while their device footprint fits
//      the arena and the per-step candidate capacity (a job that does not fit
//      waits; later arrivals wait behind it);
//   3. advance every resident job by one optimizer step with one batched
//      launch (grasp_batch_step, graph-replayed on the scheduler's stream);
//   4. retire jobs that finished their T steps (or hit a non-finite loss):
//      final forward at r_dil = 0, results and ranking copied to the host,
//      device memory freed.
// grasp_poll hands results to the caller. Every candidate is computed by the
// same per-candidate code as the single-job step, so a job's results do not
// depend on which other jobs shared its steps.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "batch.h"
#include "gs.h"

using namespace grasp;

namespace grasp {

namespace {

enum class JobState { Queued, Resident, Ended };

struct Job {
  uint64_t id = 0;
  grasp_job_desc desc{};
  std::vector<float> q0;
  int n_dof = 0;
  int n_contacts = 0;
  JobState state = JobState::Queued;
  bool cancel = false;
  grasp_status status = GRASP_OK;
  size_t footprint = 0;
  void* block = nullptr;
  float *q = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr, *terms = nullptr;
  float *metrics = nullptr, *mean = nullptr;  // evaluation at retirement (jobs with an evaluation set)
  int32_t* top = nullptr;
  float* starts = nullptr;  // Gauss-Seidel jobs: the sweep start-pose table
  size_t start_floats = 0;
  int t = 0;
  std::vector<float> out_q, out_loss, out_terms, out_metrics, out_mean;
  std::vector<int32_t> rank, out_top;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

// q, m, v, loss, terms; with an evaluation set, the metrics [B][M], the top
// indices and their mean metrics; last, a Gauss-Seidel job's start poses.
size_t job_footprint(int B, int n_dof, int M, int top_k, size_t start_floats) {
  const size_t b = static_cast<size_t>(B);
  auto r = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t f = 3 * r(b * n_dof * 4) + r(b * 4) + r(b * 16);
  if (M > 0) f += r(b * M * 4) + r(static_cast<size_t>(top_k) * 4) + r(static_cast<size_t>(M) * 4);
  return f + r(start_floats * 4);
}

int job_metrics(const grasp_job_desc& d) { return d.eval ? d.n_thr + 1 : 0; }

}  // namespace

struct Scheduler {
  grasp_ctx* ctx = nullptr;
  int32_t capacity = 65536;
  int32_t max_jobs = 256;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  bool started = false;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> resident;
  uint64_t next_id = 1;
  int64_t steps = 0, evals = 0;
  int32_t finished = 0;
  grasp_batch* batch = nullptr;
  hipStream_t stream = nullptr;
  grasp_status fatal = GRASP_OK;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - ctx->t0).count();
  }
  void run();
  bool admit_one(Job& j);
  void release(Job& j);
  void finish(Job& j);
};

void Scheduler::release(Job& j) {
  if (j.block) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->arena.free(j.block);
    j.block = nullptr;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (DevHand* h = find_hand(ctx, j.desc.hand)) h->live_jobs--;
  if (DevSdf* s = find_sdf(ctx, j.desc.sdf)) s->live_jobs--;
  if (j.desc.eval) {
    auto it = ctx->evals.find(j.desc.eval);
    if (it != ctx->evals.end()) it->second->live_jobs--;
  }
}

bool Scheduler::admit_one(Job& j) {
  void* blk = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    blk = ctx->arena.alloc(j.footprint);
  }
  if (!blk) return false;
  const size_t b = static_cast<size_t>(j.desc.B);
  auto r = [](size_t x) { return (x + 255) / 256 * 256; };
  char* p = static_cast<char*>(blk);
  const size_t nq = r(b * j.n_dof * 4);
  j.block = blk;
  j.q = reinterpret_cast<float*>(p);
  j.m = reinterpret_cast<float*>(p + nq);
  j.v = reinterpret_cast<float*>(p + 2 * nq);
  j.loss = reinterpret_cast<float*>(p + 3 * nq);
  j.terms = reinterpret_cast<float*>(p + 3 * nq + r(b * 4));
  if (const int M = job_metrics(j.desc); M > 0) {
    char* e = p + 3 * nq + r(b * 4) + r(b * 16);
    j.metrics = reinterpret_cast<float*>(e);
    j.top = reinterpret_cast<int32_t*>(e + r(b * M * 4));
    j.mean = reinterpret_cast<float*>(e + r(b * M * 4) + r(static_cast<size_t>(j.desc.top_k) * 4));
  }
  if (j.start_floats)
    j.starts = reinterpret_cast<float*>(
        p + job_footprint(j.desc.B, j.n_dof, job_metrics(j.desc), j.desc.eval ? j.desc.top_k : 0, 0));
  hipError_t e = hipMemcpyAsync(j.q, j.q0.data(), b * j.n_dof * 4, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemsetAsync(j.m, 0, 2 * nq, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    fatal = device_fail(ctx, e, "scheduler admission");
    return false;
  }
  j.q0.clear();
  j.q0.shrink_to_fit();
  j.state = JobState::Resident;
  j.t_admit = now();
  return true;
}

// Final forward at r_dil = 0, results to the host, ranking.
void Scheduler::finish(Job& j) {
  const int B = j.desc.B;
  if (j.status == GRASP_OK) {
    grasp_step_params p = j.desc.p;
    p.r_dil = 0.0f;
    p.mode = GRASP_MODE_RECOMPUTE;
    grasp_status st = grasp_step_fwd(ctx, j.desc.hand, j.desc.sdf, &p, B, j.q, j.loss, j.terms, nullptr, 0, stream);
    // post-synthesis evaluation at the final configurations, then the best by final loss
    if (st == GRASP_OK && j.metrics)
      st = grasp_evaluate(ctx, j.desc.eval, j.desc.sdf, B, j.q, j.desc.n_thr, j.desc.thresholds, j.metrics, stream);
    if (st == GRASP_OK && j.metrics && j.desc.top_k > 0)
      st = grasp_select_top(ctx, B, j.loss, 0, j.desc.top_k, j.desc.n_thr + 1, j.metrics, j.top, j.mean, stream);
    if (st != GRASP_OK) j.status = st;
  }
  if (j.state == JobState::Resident) {
    j.out_q.resize(static_cast<size_t>(B) * j.n_dof);
    j.out_loss.resize(B);
    j.out_terms.resize(static_cast<size_t>(B) * 4);
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(j.out_q.data(), j.q, j.out_q.size() * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(j.out_loss.data(), j.loss, j.out_loss.size() * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(j.out_terms.data(), j.terms, j.out_terms.size() * 4, hipMemcpyDeviceToHost);
    if (j.metrics && j.status == GRASP_OK) {
      const size_t M = static_cast<size_t>(j.desc.n_thr) + 1;
      j.out_metrics.resize(static_cast<size_t>(B) * M);
      if (e == hipSuccess) e = hipMemcpy(j.out_metrics.data(), j.metrics, j.out_metrics.size() * 4, hipMemcpyDeviceToHost);
      if (j.desc.top_k > 0) {
        j.out_top.resize(j.desc.top_k);
        j.out_mean.resize(M);
        if (e == hipSuccess) e = hipMemcpy(j.out_top.data(), j.top, j.out_top.size() * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(j.out_mean.data(), j.mean, M * 4, hipMemcpyDeviceToHost);
      }
    }
    if (e != hipSuccess) {
      fatal = device_fail(ctx, e, "scheduler results");
      j.status = GRASP_EDEVICE;
    }
    if (j.status == GRASP_OK)
      for (float x : j.out_loss)
        if (!std::isfinite(x)) j.status = GRASP_ENONFINITE;
    j.rank.resize(B);
    std::iota(j.rank.begin(), j.rank.end(), 0);
    std::stable_sort(j.rank.begin(), j.rank.end(), [&](int a, int b) { return j.out_loss[a] < j.out_loss[b]; });
  }
  release(j);
  j.state = JobState::Ended;
  j.t_done = now();
}

void Scheduler::run() {
  (void)hipSetDevice(ctx->device);
  std::vector<grasp_batch_job> bj;
  std::vector<Job*> bjob, gsjob;
  std::vector<int32_t> flags;
  std::vector<grasp_status> gs_st;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      // 1. cancellations
      for (auto it = queue.begin(); it != queue.end();) {
        Job& j = *jobs[*it];
        if (j.cancel) {
          j.status = GRASP_ECANCELED;
          release(j);
          j.state = JobState::Ended;
          j.t_done = now();
          ++finished;
          it = queue.erase(it);
        } else {
          ++it;
        }
      }
      for (auto it = resident.begin(); it != resident.end();) {
        Job& j = *jobs[*it];
        if (j.cancel) {
          j.status = GRASP_ECANCELED;
          j.state = JobState::Ended;  // results are not copied for a cancelled job
          release(j);
          j.t_done = now();
          ++finished;
          it = resident.erase(it);
        } else {
          ++it;
        }
      }
      cv.notify_all();
      // 2. admission, first come first served
      int64_t cand = 0;
      for (uint64_t id : resident) cand += jobs[id]->desc.B;
      while (!queue.empty() && fatal == GRASP_OK && static_cast<int32_t>(resident.size()) < max_jobs) {
        Job& j = *jobs[queue.front()];
        if (cand + j.desc.B > capacity) break;
        if (!admit_one(j)) break;
        cand += j.desc.B;
        resident.push_back(j.id);
        queue.pop_front();
      }
      if (stop && queue.empty() && resident.empty()) return;
      if (stop || fatal != GRASP_OK) {
        // shutting down or poisoned: end everything
        for (uint64_t id : queue) {
          Job& j = *jobs[id];
          j.status = fatal != GRASP_OK ? fatal : GRASP_ECANCELED;
          release(j);
          j.state = JobState::Ended;
          ++finished;
        }
        queue.clear();
        for (uint64_t id : resident) {
          Job& j = *jobs[id];
          j.status = fatal != GRASP_OK ? fatal : GRASP_ECANCELED;
          release(j);
          j.state = JobState::Ended;
          ++finished;
        }
        resident.clear();
        cv.notify_all();
        return;
      }
      if (resident.empty()) {
        cv.wait_for(lk, std::chrono::milliseconds(50));
        continue;
      }
      bj.clear();
      bjob.clear();
      gsjob.clear();
      for (uint64_t id : resident) {
        Job& j = *jobs[id];
        if (j.desc.p.projection == GRASP_PROJECTION_GAUSS_SEIDEL) {
          gsjob.push_back(&j);  // stepped by a launch of its own
          continue;
        }
        grasp_batch_job b{};
        b.hand = j.desc.hand;
        b.sdf = j.desc.sdf;
        b.p = j.desc.p;
        b.B = j.desc.B;
        b.q = j.q;
        b.m = j.m;
        b.v = j.v;
        b.loss = j.loss;
        b.terms = nullptr;
        b.t = j.t;
        b.T = j.desc.T;
        b.r0 = j.desc.r0;
        b.lr = j.desc.lr;
        b.b1 = j.desc.b1;
        b.b2 = j.desc.b2;
        b.eps = j.desc.eps;
        bj.push_back(b);
        bjob.push_back(&j);
      }
    }
    // 3. one batched step for every resident job (outside the lock); a
    // Gauss-Seidel job's sweep is its own fused launch on the same stream,
    // with the same dilation schedule and its own start-pose table
    grasp_status st = GRASP_OK;
    flags.assign(bj.size(), 0);
    if (!bj.empty()) {
      st = grasp_batch_step(batch, bj.data(), static_cast<int32_t>(bj.size()), stream);
      if (st == GRASP_OK) st = grasp_batch_flags(batch, static_cast<int32_t>(bj.size()), flags.data());
    }
    gs_st.assign(gsjob.size(), GRASP_OK);
    for (size_t k = 0; k < gsjob.size() && st == GRASP_OK; ++k) {
      Job* j = gsjob[k];
      grasp_step_params p = j->desc.p;
      p.r_dil = dilation_at(j->desc.r0, j->t, j->desc.T);
      // a refusal ends this job only
      gs_st[k] = step_fused_gs(ctx, j->desc.hand, j->desc.sdf, &p, j->desc.B, j->q, j->m, j->v, j->t + 1, j->desc.lr,
                               j->desc.b1, j->desc.b2, j->desc.eps, j->loss, j->starts, stream);
      if (gs_st[k] == GRASP_EDEVICE) st = GRASP_EDEVICE;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      if (st != GRASP_OK) {
        fatal = st;
        continue;
      }
      ++steps;
      for (size_t k = 0; k < bj.size(); ++k) {
        Job& j = *bjob[k];
        j.t = bj[k].t;
        evals += static_cast<int64_t>(j.desc.B) * j.n_contacts * 7 * j.desc.p.K;
        if (flags[k]) j.status = GRASP_ENONFINITE;
      }
      for (size_t k = 0; k < gsjob.size(); ++k) {
        Job& j = *gsjob[k];
        if (gs_st[k] != GRASP_OK) {
          j.status = gs_st[k];
          continue;
        }
        ++j.t;
        evals += static_cast<int64_t>(j.desc.B) * j.n_contacts * 7 * j.desc.p.K;
      }
      // 4. retire finished jobs
      for (auto it = resident.begin(); it != resident.end();) {
        Job& j = *jobs[*it];
        if (j.t >= j.desc.T || j.status != GRASP_OK) {
          finish(j);
          ++finished;
          it = resident.erase(it);
        } else {
          ++it;
        }
      }
      cv.notify_all();
    }
  }
}

}  // namespace grasp

namespace {

Scheduler* sched_of(grasp_ctx* ctx, bool create, grasp_status* st) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->sched || !create) return ctx->sched;
  auto* s = new Scheduler();
  s->ctx = ctx;
  ctx->sched = s;
  *st = GRASP_OK;
  return s;
}

grasp_status start(Scheduler* s) {
  if (s->started) return GRASP_OK;
  DeviceGuard g(s->ctx->device);
  hipError_t e = hipStreamCreate(&s->stream);
  if (e != hipSuccess) return device_fail(s->ctx, e, "scheduler stream");
  grasp_status st = grasp_batch_create(s->ctx, s->capacity, s->max_jobs, 1, &s->batch);
  if (st != GRASP_OK) return st;
  s->started = true;
  s->th = std::thread([s] { s->run(); });
  return GRASP_OK;
}

}  // namespace

extern "C" {

void grasp_shutdown_scheduler(grasp_ctx* ctx) {
  if (!ctx || !ctx->sched) return;
  Scheduler* s = ctx->sched;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto& kv : s->jobs) kv.second->cancel = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  {
    DeviceGuard g(ctx->device);
    if (s->batch) grasp_batch_destroy(s->batch);
    if (s->stream) (void)hipStreamDestroy(s->stream);
  }
  delete s;
  ctx->sched = nullptr;
}

grasp_status grasp_serve_config(grasp_ctx* ctx, int32_t capacity, int32_t max_jobs) {
  set_error("");
  if (!ctx) return fail(GRASP_EINVAL, "context is NULL");
  if (capacity < 1 || max_jobs < 1 || max_jobs > 4096) return fail(GRASP_EINVAL, "bad capacity / max_jobs");
  grasp_status st = GRASP_OK;
  Scheduler* s = sched_of(ctx, true, &st);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->started) return fail(GRASP_EBUSY, "the scheduler is already running");
  s->capacity = capacity;
  s->max_jobs = max_jobs;
  return GRASP_OK;
}

grasp_status grasp_submit(grasp_ctx* ctx, const grasp_job_desc* d, grasp_job_id* out) {
  set_error("");
  if (!ctx || !d || !out) return fail(GRASP_EINVAL, "ctx/job/out is NULL");
  if (ctx->poisoned) return fail(GRASP_EDEVICE, "context poisoned");
  if (d->B < 1 || !d->q0 || d->T < 1 || !(d->r0 >= 0.0f)) return fail(GRASP_EINVAL, "job needs B >= 1, q0, T >= 1, r0 >= 0");
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
    if (d->top_k < 0 || d->top_k > std::min(d->B, GRASP_MAX_TOP)) return fail(GRASP_EINVAL, "top_k must be in [0, min(B, 64)]");
  } else if (d->top_k != 0) {
    return fail(GRASP_EINVAL, "top_k needs an evaluation set");
  }
  st = GRASP_OK;
  Scheduler* s = sched_of(ctx, true, &st);
  auto j = std::make_unique<Job>();
  j->desc = *d;
  j->n_dof = n_dof;
  j->n_contacts = nc;
  // a Gauss-Seidel job keeps its own start-pose table, reserved at admission
  j->start_floats = d->p.projection == GRASP_PROJECTION_GAUSS_SEIDEL ? gs_scratch_floats(d->B, hv.n_chunks, d->p.K) : 0;
  j->footprint = job_footprint(d->B, n_dof, job_metrics(*d), d->eval ? d->top_k : 0, j->start_floats);
  j->q0.assign(d->q0, d->q0 + static_cast<size_t>(d->B) * n_dof);
  j->desc.q0 = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (d->B > s->capacity || j->footprint > ctx->arena.capacity())
      return fail(GRASP_ENOMEM, "job can never fit the candidate capacity or the arena");
    st = start(s);
    if (st != GRASP_OK) return st;
    {
      std::lock_guard<std::mutex> lk2(ctx->mu);
      DevEval* ev = nullptr;
      if (d->eval) {
        auto it = ctx->evals.find(d->eval);
        if (it == ctx->evals.end()) return fail(GRASP_EINVAL, "unknown evaluation set id");
        ev = it->second.get();
      }
      find_hand(ctx, d->hand)->live_jobs++;
      find_sdf(ctx, d->sdf)->live_jobs++;
      if (ev) ev->live_jobs++;
    }
    j->id = s->next_id++;
    j->t_submit = s->now();
    *out = j->id;
    s->queue.push_back(j->id);
    s->jobs[j->id] = std::move(j);
  }
  s->cv.notify_all();
  return GRASP_OK;
}

grasp_status grasp_poll(grasp_ctx* ctx, grasp_job_id id, grasp_job_result* r) {
  set_error("");
  if (!ctx || !r) return fail(GRASP_EINVAL, "ctx/result is NULL");
  Scheduler* s = ctx->sched;
  if (!s) return fail(GRASP_EINVAL, "unknown job id");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return fail(GRASP_EINVAL, "unknown job id");
  Job& j = *it->second;
  if (j.state != JobState::Ended) return GRASP_EAGAIN;
  const int B = j.desc.B;
  if (!j.out_q.empty()) {
    if (r->q) std::memcpy(r->q, j.out_q.data(), j.out_q.size() * 4);
    if (r->loss) std::memcpy(r->loss, j.out_loss.data(), static_cast<size_t>(B) * 4);
    if (r->terms) std::memcpy(r->terms, j.out_terms.data(), static_cast<size_t>(B) * 16);
    if (r->rank) std::memcpy(r->rank, j.rank.data(), static_cast<size_t>(B) * 4);
    if (r->metrics && !j.out_metrics.empty()) std::memcpy(r->metrics, j.out_metrics.data(), j.out_metrics.size() * 4);
    if (r->top && !j.out_top.empty()) std::memcpy(r->top, j.out_top.data(), j.out_top.size() * 4);
    if (r->top_mean && !j.out_mean.empty()) std::memcpy(r->top_mean, j.out_mean.data(), j.out_mean.size() * 4);
  }
  r->status = j.status;
  r->t_submit = j.t_submit;
  r->t_admit = j.t_admit;
  r->t_done = j.t_done;
  r->steps = j.t;
  const grasp_status st = j.status;
  s->jobs.erase(it);
  if (st != GRASP_OK) set_error("job ended with a non-OK status");
  return st;
}

grasp_status grasp_cancel(grasp_ctx* ctx, grasp_job_id id) {
  set_error("");
  if (!ctx || !ctx->sched) return fail(GRASP_EINVAL, "unknown job id");
  Scheduler* s = ctx->sched;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return fail(GRASP_EINVAL, "unknown job id");
    it->second->cancel = true;
  }
  s->cv.notify_all();
  return GRASP_OK;
}

grasp_status grasp_serve_stats_get(grasp_ctx* ctx, grasp_serve_stats* out) {
  set_error("");
  if (!ctx || !out) return fail(GRASP_EINVAL, "ctx/out is NULL");
  std::memset(out, 0, sizeof(*out));
  Scheduler* s = ctx->sched;
  if (!s) return GRASP_OK;
  std::lock_guard<std::mutex> lk(s->mu);
  out->steps = s->steps;
  out->contact_evals = s->evals;
  out->queued = static_cast<int32_t>(s->queue.size());
  out->resident = static_cast<int32_t>(s->resident.size());
  out->finished = s->finished;
  return GRASP_OK;
}

}  // extern "C"
