// Serving loop of the grasp library, host part: the job queue, admission at
// step boundaries, one step of every resident job at a time, retirement,
// cancellation and the scheduler thread. What a job does on the device
// (memory, steps, final forward, results) goes through a ServeExecutor, so
// the loop itself is plain C++ with no HIP in it and is tested on the CPU
// with an executor that computes on the host.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "grasp.h"

namespace grasp {

enum class JobState { Queued, Resident, Ended };

struct ServeJob {
  uint64_t id = 0;
  grasp_job_desc desc{};       // desc.q0 is cleared; the start lives in q0
  std::vector<float> q0;       // [B][n_dof] until admission
  int n_dof = 0;
  int n_contacts = 0;
  size_t footprint = 0;        // device bytes the executor needs while the job is resident
  JobState state = JobState::Queued;
  bool cancel = false;
  grasp_status status = GRASP_OK;
  int t = 0;                   // optimizer steps taken
  double t_submit = 0, t_admit = 0, t_done = 0;
  // results, filled by the executor's finish
  std::vector<float> out_q, out_loss, out_terms, out_metrics, out_mean;
  std::vector<int32_t> rank, out_top;
  // with desc.record_history: q before and loss at each step, [T][B][n_dof] and [T][B]
  std::vector<float> hist_q, hist_loss;
  void* exec = nullptr;        // the executor's per-job state
};

// Device side of the loop. Every call comes from the scheduler thread, one at
// a time. An exception thrown by any call is a fatal error of the loop: every
// job still queued or resident ends with GRASP_EDEVICE and later submissions
// are refused.
class ServeExecutor {
 public:
  virtual ~ServeExecutor() = default;
  // Reserves the job's memory and uploads its start: GRASP_OK (resident),
  // GRASP_EAGAIN (no room now: the job waits, and so do later arrivals), or a
  // fatal status.
  virtual grasp_status admit(ServeJob& j) = 0;
  // One optimizer step of every job in `jobs` (each advances t by one);
  // st[k] gets the job's own status (GRASP_OK, GRASP_ENONFINITE, or an error
  // that ends that job only). Returns a fatal status or GRASP_OK. When it
  // returns, the step's results are visible to the host.
  virtual grasp_status step(const std::vector<ServeJob*>& jobs, std::vector<grasp_status>& st) = 0;
  // Final results of a resident job into its out_* vectors; may change its
  // status (ENONFINITE, EDEVICE).
  virtual void finish(ServeJob& j) = 0;
  // Waits until no device work of any job is in flight.
  virtual void drain() = 0;
  // Gives back whatever the job holds (its memory if resident; references to
  // its hand, grid and evaluation set). Called once per job, after drain()
  // for a resident job.
  virtual void release(ServeJob& j) = 0;
};

class ServeLoop {
 public:
  // clock: seconds since an epoch shared with the caller.
  ServeLoop(ServeExecutor* ex, std::function<double()> clock) : ex_(ex), clock_(std::move(clock)) {}
  ~ServeLoop() { shutdown(); }

  // Candidate capacity per step and job limit; only before the first submit.
  grasp_status configure(int32_t capacity, int32_t max_jobs);
  int32_t capacity() const { return capacity_; }
  // Queues a job; arena_capacity is the most device memory it could ever get.
  // ENOMEM when it can never fit; EDEVICE after a fatal error. Starts the
  // thread on first use. on_accept runs under the loop's lock just before the
  // job is queued (the caller takes its references there).
  grasp_status submit(std::unique_ptr<ServeJob> j, size_t arena_capacity, const std::function<void()>& on_accept,
                      uint64_t* out);
  grasp_status poll(uint64_t id, grasp_job_result* r);
  grasp_status cancel(uint64_t id);
  void stats(grasp_serve_stats* out);
  // Ends every job (cancelled), stops and joins the thread.
  void shutdown();

 private:
  void run();
  void end_job(ServeJob& j, grasp_status st);
  void fail_all(grasp_status st);

  ServeExecutor* ex_;
  std::function<double()> clock_;
  int32_t capacity_ = 65536;
  int32_t max_jobs_ = 256;
  std::thread th_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
  bool started_ = false;
  grasp_status fatal_ = GRASP_OK;
  std::map<uint64_t, std::unique_ptr<ServeJob>> jobs_;
  std::deque<uint64_t> queue_;
  std::vector<uint64_t> resident_;
  uint64_t next_id_ = 1;
  int64_t steps_ = 0, evals_ = 0;
  int32_t finished_ = 0;
};

// Candidate indices by ascending final loss, NaN after every number, ties by
// index (a stable sort).
std::vector<int32_t> rank_by_loss(const std::vector<float>& loss);

}  // namespace grasp
