// Serving loop core (see serve_core.h). The scheduler thread repeats, at
// every step boundary:
//   1. end cancelled jobs (queued ones at once; resident ones after the
//      device has finished their last step);
//   2. admit queued jobs in arrival order while the candidate capacity, the
//      job limit and the executor's memory allow (a job that does not fit
//      waits; later arrivals wait behind it);
//   3. advance every resident job by one optimizer step (one executor call);
//   4. retire jobs that took their T steps or whose step failed.
// Job state is guarded by one mutex; executor calls that touch the device run
// outside it, on resident jobs only, which nothing else modifies meanwhile.
#include "serve_core.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <numeric>

namespace grasp {

std::vector<int32_t> rank_by_loss(const std::vector<float>& loss) {
  std::vector<int32_t> r(loss.size());
  std::iota(r.begin(), r.end(), 0);
  std::stable_sort(r.begin(), r.end(), [&](int32_t a, int32_t b) {
    const bool na = std::isnan(loss[a]), nb = std::isnan(loss[b]);
    if (na != nb) return nb;  // numbers before NaN
    return !na && loss[a] < loss[b];
  });
  return r;
}

grasp_status ServeLoop::configure(int32_t capacity, int32_t max_jobs) {
  if (capacity < 1 || max_jobs < 1 || max_jobs > 4096) return GRASP_EINVAL;
  std::lock_guard<std::mutex> lk(mu_);
  if (started_) return GRASP_EBUSY;
  capacity_ = capacity;
  max_jobs_ = max_jobs;
  return GRASP_OK;
}

grasp_status ServeLoop::submit(std::unique_ptr<ServeJob> j, size_t arena_capacity,
                               const std::function<void()>& on_accept, uint64_t* out) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (fatal_ != GRASP_OK) return GRASP_EDEVICE;
    if (stop_) return GRASP_EINVAL;
    if (j->desc.B > capacity_ || j->footprint > arena_capacity) return GRASP_ENOMEM;
    if (!started_) {
      started_ = true;
      th_ = std::thread([this] { run(); });
    }
    if (on_accept) on_accept();
    j->id = next_id_++;
    j->t_submit = clock_();
    j->state = JobState::Queued;
    *out = j->id;
    queue_.push_back(j->id);
    jobs_[j->id] = std::move(j);
  }
  cv_.notify_all();
  return GRASP_OK;
}

grasp_status ServeLoop::poll(uint64_t id, grasp_job_result* r) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = jobs_.find(id);
  if (it == jobs_.end()) return GRASP_EINVAL;
  ServeJob& j = *it->second;
  if (j.state != JobState::Ended) return GRASP_EAGAIN;
  const size_t B = static_cast<size_t>(j.desc.B);
  if (!j.out_q.empty()) {
    if (r->q) std::memcpy(r->q, j.out_q.data(), j.out_q.size() * 4);
    if (r->loss) std::memcpy(r->loss, j.out_loss.data(), B * 4);
    if (r->terms) std::memcpy(r->terms, j.out_terms.data(), B * 16);
    if (r->rank) std::memcpy(r->rank, j.rank.data(), B * 4);
    if (r->metrics && !j.out_metrics.empty()) std::memcpy(r->metrics, j.out_metrics.data(), j.out_metrics.size() * 4);
    if (r->top && !j.out_top.empty()) std::memcpy(r->top, j.out_top.data(), j.out_top.size() * 4);
    if (r->top_mean && !j.out_mean.empty()) std::memcpy(r->top_mean, j.out_mean.data(), j.out_mean.size() * 4);
  }
  // history of the steps taken (the rest of the caller's [T] rows untouched)
  if (r->hist_q && !j.hist_q.empty())
    std::memcpy(r->hist_q, j.hist_q.data(), static_cast<size_t>(j.t) * B * j.n_dof * 4);
  if (r->hist_loss && !j.hist_loss.empty())
    std::memcpy(r->hist_loss, j.hist_loss.data(), static_cast<size_t>(j.t) * B * 4);
  r->status = j.status;
  r->t_submit = j.t_submit;
  r->t_admit = j.t_admit;
  r->t_done = j.t_done;
  r->steps = j.t;
  const grasp_status st = j.status;
  jobs_.erase(it);
  return st;
}

grasp_status ServeLoop::cancel(uint64_t id) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(id);
    if (it == jobs_.end()) return GRASP_EINVAL;
    it->second->cancel = true;
  }
  cv_.notify_all();
  return GRASP_OK;
}

void ServeLoop::stats(grasp_serve_stats* out) {
  std::lock_guard<std::mutex> lk(mu_);
  out->steps = steps_;
  out->contact_evals = evals_;
  out->queued = static_cast<int32_t>(queue_.size());
  out->resident = static_cast<int32_t>(resident_.size());
  out->finished = finished_;
}

void ServeLoop::shutdown() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
    for (auto& kv : jobs_) kv.second->cancel = true;
  }
  cv_.notify_all();
  if (th_.joinable()) th_.join();
}

// Caller holds mu_. The job's device work has finished (queued, or drained).
void ServeLoop::end_job(ServeJob& j, grasp_status st) {
  if (st != GRASP_OK) j.status = st;
  try {
    ex_->release(j);
  } catch (...) {
    fatal_ = GRASP_EDEVICE;
  }
  j.state = JobState::Ended;
  j.t_done = clock_();
  ++finished_;
}

// Caller holds mu_: ends every queued and resident job with st.
void ServeLoop::fail_all(grasp_status st) {
  if (!resident_.empty()) {
    try {
      ex_->drain();
    } catch (...) {
    }
  }
  for (uint64_t id : queue_) end_job(*jobs_[id], st);
  queue_.clear();
  for (uint64_t id : resident_) end_job(*jobs_[id], st);
  resident_.clear();
}

void ServeLoop::run() {
  std::vector<ServeJob*> step_jobs;
  std::vector<grasp_status> st;
  std::unique_lock<std::mutex> lk(mu_);
  for (;;) {
    // 1. cancellations
    for (auto it = queue_.begin(); it != queue_.end();) {
      ServeJob& j = *jobs_[*it];
      if (j.cancel) {
        end_job(j, GRASP_ECANCELED);
        it = queue_.erase(it);
      } else {
        ++it;
      }
    }
    bool drained = false;
    for (auto it = resident_.begin(); it != resident_.end();) {
      ServeJob& j = *jobs_[*it];
      if (j.cancel) {
        if (!drained) {
          // the job's memory may still be read by its last step
          try {
            ex_->drain();
          } catch (...) {
            fatal_ = GRASP_EDEVICE;
          }
          drained = true;
        }
        end_job(j, GRASP_ECANCELED);  // results are not copied for a cancelled job
        it = resident_.erase(it);
      } else {
        ++it;
      }
    }
    cv_.notify_all();
    // 2. admission, first come first served
    int64_t cand = 0;
    for (uint64_t id : resident_) cand += jobs_[id]->desc.B;
    while (!queue_.empty() && fatal_ == GRASP_OK && static_cast<int32_t>(resident_.size()) < max_jobs_) {
      ServeJob& j = *jobs_[queue_.front()];
      if (cand + j.desc.B > capacity_) break;
      grasp_status a;
      try {
        a = ex_->admit(j);
      } catch (...) {
        a = GRASP_EDEVICE;
      }
      if (a == GRASP_EAGAIN) break;
      if (a != GRASP_OK) {
        fatal_ = a;
        break;
      }
      j.state = JobState::Resident;
      j.t_admit = clock_();
      j.q0.clear();
      j.q0.shrink_to_fit();
      cand += j.desc.B;
      resident_.push_back(j.id);
      queue_.pop_front();
    }
    if (fatal_ != GRASP_OK || stop_) {
      // poisoned or shutting down: end everything still here
      fail_all(fatal_ != GRASP_OK ? fatal_ : GRASP_ECANCELED);
      cv_.notify_all();
      return;
    }
    if (resident_.empty()) {
      // a system-clock deadline waits through pthread_cond_timedwait, which
      // thread sanitizers see; a clock jump only shortens or lengthens one nap
      cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(50));
      continue;
    }
    // 3. one step of every resident job, outside the lock
    step_jobs.clear();
    for (uint64_t id : resident_) step_jobs.push_back(jobs_[id].get());
    st.assign(step_jobs.size(), GRASP_OK);
    lk.unlock();
    grasp_status s;
    try {
      s = ex_->step(step_jobs, st);
    } catch (...) {
      s = GRASP_EDEVICE;
    }
    lk.lock();
    if (s != GRASP_OK) {
      fatal_ = s;
      continue;
    }
    ++steps_;
    for (size_t k = 0; k < step_jobs.size(); ++k) {
      ServeJob& j = *step_jobs[k];
      if (st[k] == GRASP_OK || st[k] == GRASP_ENONFINITE) {
        ++j.t;
        evals_ += static_cast<int64_t>(j.desc.B) * j.n_contacts * 7 * j.desc.p.K;
      }
      if (st[k] != GRASP_OK) j.status = st[k];
    }
    // 4. retire finished jobs
    for (auto it = resident_.begin(); it != resident_.end();) {
      ServeJob& j = *jobs_[*it];
      if (j.t >= j.desc.T || j.status != GRASP_OK) {
        try {
          ex_->finish(j);
          ex_->drain();
        } catch (...) {
          j.status = GRASP_EDEVICE;
          fatal_ = GRASP_EDEVICE;
        }
        end_job(j, GRASP_OK);
        it = resident_.erase(it);
      } else {
        ++it;
      }
    }
    cv_.notify_all();
  }
}

}  // namespace grasp
