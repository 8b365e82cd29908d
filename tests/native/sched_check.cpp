// The serving loop's host core (serve_core.cpp) driven by an executor that
// computes on the CPU: each job's memory comes from an Arena over a host
// buffer (admission by footprint), and each optimizer step is the FP64
// oracle's step and Adam on the job's own state (the oracle as a test
// double for the device). Built with ThreadSanitizer by the test suite.
//
// Checks: concurrent submit / poll / cancel from several threads; every job
// ends exactly once with a consistent status; a completed job's results equal
// the same job run alone, bit for bit; admission under a full arena (a job
// waits until memory frees, then runs); the job limit; a job that can never
// fit is refused; an executor that throws ends every live job with
// GRASP_EDEVICE and refuses later submissions; shutdown with jobs in flight.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <random>
#include <stdexcept>
#include <thread>
#include <vector>

#include "arena.h"
#include "oracle_api.h"
#include "serve_core.h"

using namespace grasp;

namespace {

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::printf("check failed: %s (line %d)\n", #c, __LINE__);        \
      std::exit(1);                                                     \
    }                                                                   \
  } while (0)

// A palm-only hand with four contacts and a sphere of radius 4 cm.
struct Problem {
  int parent[1] = {-1};
  double origin[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
  double axis[3] = {0, 0, 1};
  double qlo[6] = {0, 0, 0, 0, 0, 0}, qup[6] = {0, 0, 0, 0, 0, 0};
  double local[12] = {0.0, 0.0, -0.039, 0.01, 0.0, -0.0395, -0.01, 0.005, -0.0385, 0.0, -0.01, -0.041};
  int link[4] = {0, 0, 0, 0};
  ohand hand{};
  oobject obj{};
  Problem() {
    hand = ohand{1, parent, origin, axis, qlo, qup, 4, local, link};
    std::memset(&obj, 0, sizeof(obj));
    obj.kind = OBJ_SPHERE;
    obj.radius = 0.04;
    obj.inertia_over_mass = 0.4 * 0.04 * 0.04;
  }
};
const Problem& problem() {
  static Problem p;
  return p;
}

constexpr int kDof = 6;

struct HostJob {
  void* block = nullptr;
  std::vector<double> q, m, v;
};

// The CPU executor. mu_ guards the arena, which release() (under the loop's
// lock) and admit() (under the loop's lock) share with nothing else; the
// counters check the loop's calling discipline.
class CpuExecutor final : public ServeExecutor {
 public:
  CpuExecutor(size_t arena_bytes, int throw_at_step = -1) : storage_(arena_bytes + 256), throw_at_(throw_at_step) {
    char* base = storage_.data();
    base += (256 - reinterpret_cast<uintptr_t>(base) % 256) % 256;
    arena_.reset(base, arena_bytes);
  }
  size_t capacity() const { return arena_.capacity(); }

  grasp_status admit(ServeJob& j) override {
    CHECK(in_call_.exchange(true) == false);
    void* blk = arena_.alloc(j.footprint);
    if (!blk) {
      in_call_ = false;
      return GRASP_EAGAIN;
    }
    auto* h = new HostJob();
    h->block = blk;
    h->q.assign(j.q0.begin(), j.q0.end());
    h->m.assign(j.q0.size(), 0.0);
    h->v.assign(j.q0.size(), 0.0);
    CHECK(j.exec == nullptr);
    j.exec = h;
    ++admitted_;
    const int live = ++resident_;
    if (live > max_resident_) max_resident_ = live;
    in_call_ = false;
    return GRASP_OK;
  }

  grasp_status step(const std::vector<ServeJob*>& jobs, std::vector<grasp_status>& st) override {
    CHECK(in_call_.exchange(true) == false);
    if (throw_at_ >= 0 && steps_ == throw_at_) {
      in_call_ = false;
      throw std::runtime_error("executor failure");
    }
    ++steps_;
    for (size_t k = 0; k < jobs.size(); ++k) {
      ServeJob& j = *jobs[k];
      CHECK(j.state == JobState::Resident && j.exec);
      st[k] = step_job(j);
    }
    in_call_ = false;
    return GRASP_OK;
  }

  void finish(ServeJob& j) override {
    CHECK(in_call_.exchange(true) == false);
    auto* h = static_cast<HostJob*>(j.exec);
    const int B = j.desc.B;
    std::vector<double> loss(B), terms(4 * B);
    oparams P = params(0.0);
    CHECK(oracle_step(&problem().hand, &problem().obj, &P, B, h->q.data(), loss.data(), terms.data(), nullptr,
                      nullptr, 1) == 0);
    j.out_q.assign(h->q.begin(), h->q.end());
    j.out_loss.assign(loss.begin(), loss.end());
    j.out_terms.assign(terms.begin(), terms.end());
    for (float x : j.out_loss)
      if (!std::isfinite(x)) j.status = GRASP_ENONFINITE;
    j.rank = rank_by_loss(j.out_loss);
    in_call_ = false;
  }

  void drain() override {}

  void release(ServeJob& j) override {
    auto* h = static_cast<HostJob*>(j.exec);
    if (h) {
      arena_.free(h->block);
      delete h;
      j.exec = nullptr;
      --resident_;
    }
    ++released_;
  }

  // One optimizer step of a job on the CPU (the dilation schedule of the
  // device form: r0 (1 - t / (T - 1))).
  static grasp_status step_job_state(const grasp_job_desc& d, int t, std::vector<double>& q, std::vector<double>& m,
                                     std::vector<double>& v, float* hist_loss) {
    const int B = d.B;
    const double r = d.T > 1 ? d.r0 * (1.0 - static_cast<double>(std::min(t, d.T - 1)) / (d.T - 1)) : 0.0;
    oparams P = params(r);
    std::vector<double> loss(B), grad(static_cast<size_t>(B) * kDof);
    CHECK(oracle_step(&problem().hand, &problem().obj, &P, B, q.data(), loss.data(), nullptr, grad.data(), nullptr,
                      1) == 0);
    CHECK(oracle_adam(B * kDof, q.data(), m.data(), v.data(), grad.data(), t + 1, d.lr, d.b1, d.b2, d.eps) == 0);
    bool finite = true;
    for (int b = 0; b < B; ++b) {
      if (hist_loss) hist_loss[b] = static_cast<float>(loss[b]);
      finite = finite && std::isfinite(loss[b]);
    }
    return finite ? GRASP_OK : GRASP_ENONFINITE;
  }

  static oparams params(double r) {
    oparams P{};
    P.dt = 1e-3;
    P.v0 = 1.0;
    P.K = 1;
    P.omega = 1.0;
    P.r_dil = r;
    P.alpha_leak = 0.1;
    P.w_stable = 1.0;
    P.w_pen = 1e4;
    P.w_range = 1e-2;
    P.w_limit = 1.0;
    P.w_min = 1e-8;
    P.projection = 0;
    return P;
  }

  int steps() const { return steps_; }
  int max_resident() const { return max_resident_; }
  int admitted() const { return admitted_; }
  int released() const { return released_; }

 private:
  grasp_status step_job(ServeJob& j) {
    auto* h = static_cast<HostJob*>(j.exec);
    if (j.desc.record_history) {
      if (j.hist_q.empty()) {
        j.hist_q.assign(static_cast<size_t>(j.desc.T) * j.desc.B * kDof, 0.0f);
        j.hist_loss.assign(static_cast<size_t>(j.desc.T) * j.desc.B, 0.0f);
      }
      for (size_t i = 0; i < h->q.size(); ++i)
        j.hist_q[static_cast<size_t>(j.t) * j.desc.B * kDof + i] = static_cast<float>(h->q[i]);
    }
    return step_job_state(j.desc, j.t, h->q, h->m, h->v,
                          j.desc.record_history ? j.hist_loss.data() + static_cast<size_t>(j.t) * j.desc.B : nullptr);
  }

  std::vector<char> storage_;
  Arena arena_;
  int throw_at_;
  std::atomic<bool> in_call_{false};
  int steps_ = 0, admitted_ = 0, released_ = 0;
  int resident_ = 0, max_resident_ = 0;
};

double now() {
  static const auto t0 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

grasp_job_desc make_desc(int B, int T, uint32_t seed, std::vector<float>& q0) {
  std::mt19937 rng(seed);
  std::uniform_real_distribution<float> u(-0.004f, 0.004f);
  q0.resize(static_cast<size_t>(B) * kDof);
  for (auto& x : q0) x = u(rng);
  grasp_job_desc d{};
  d.B = B;
  d.q0 = q0.data();
  d.T = T;
  d.r0 = 0.003f;
  d.lr = 1e-3f;
  d.b1 = 0.9f;
  d.b2 = 0.999f;
  d.eps = 1e-8f;
  d.p.K = 1;
  return d;
}

size_t footprint_of(int B) { return static_cast<size_t>(B) * 1024; }

std::unique_ptr<ServeJob> make_job(const grasp_job_desc& d) {
  auto j = std::make_unique<ServeJob>();
  j->desc = d;
  j->q0.assign(d.q0, d.q0 + static_cast<size_t>(d.B) * kDof);
  j->desc.q0 = nullptr;
  j->n_dof = kDof;
  j->n_contacts = 4;
  j->footprint = footprint_of(d.B);
  return j;
}

struct Result {
  grasp_status st;
  std::vector<float> q, loss, hist_loss;
  std::vector<int32_t> rank;
  int steps;
  double t_admit, t_done;
};

// Polls until the job ends.
Result wait(ServeLoop& L, uint64_t id, int B, int T) {
  Result r;
  r.q.assign(static_cast<size_t>(B) * kDof, 0.0f);
  r.loss.assign(B, 0.0f);
  r.hist_loss.assign(static_cast<size_t>(T) * B, -1.0f);
  r.rank.assign(B, -1);
  std::vector<float> terms(4 * B), hq(static_cast<size_t>(T) * B * kDof);
  for (;;) {
    grasp_job_result res{};
    res.q = r.q.data();
    res.loss = r.loss.data();
    res.terms = terms.data();
    res.rank = r.rank.data();
    res.hist_q = hq.data();
    res.hist_loss = r.hist_loss.data();
    const grasp_status st = L.poll(id, &res);
    if (st != GRASP_EAGAIN) {
      r.st = st;
      r.steps = res.steps;
      r.t_admit = res.t_admit;
      r.t_done = res.t_done;
      CHECK(res.status == st);
      return r;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

// The same job alone on the CPU: the reference a served job must equal.
std::vector<float> run_alone(const grasp_job_desc& d, const std::vector<float>& q0, std::vector<float>* hist) {
  std::vector<double> q(q0.begin(), q0.end()), m(q.size(), 0.0), v(q.size(), 0.0);
  if (hist) hist->assign(static_cast<size_t>(d.T) * d.B, 0.0f);
  for (int t = 0; t < d.T; ++t)
    CpuExecutor::step_job_state(d, t, q, m, v, hist ? hist->data() + static_cast<size_t>(t) * d.B : nullptr);
  return std::vector<float>(q.begin(), q.end());
}

void test_mix_equals_alone() {
  CpuExecutor ex(1 << 20);
  ServeLoop L(&ex, now);
  CHECK(L.configure(64, 8) == GRASP_OK);
  const int n_jobs = 24;
  std::vector<std::vector<float>> q0(n_jobs);
  std::vector<grasp_job_desc> descs(n_jobs);
  std::vector<uint64_t> ids(n_jobs, 0);
  std::vector<bool> want_cancel(n_jobs, false);
  for (int i = 0; i < n_jobs; ++i) {
    descs[i] = make_desc(1 + i % 5, 3 + i % 7, 100 + i, q0[i]);
    descs[i].record_history = i % 2;
    want_cancel[i] = i % 6 == 5;
  }
  // submitters on three threads; a canceller; pollers on two threads
  std::atomic<int> submitted{0};
  std::vector<std::thread> th;
  for (int w = 0; w < 3; ++w)
    th.emplace_back([&, w] {
      for (int i = w; i < n_jobs; i += 3) {
        uint64_t id = 0;
        CHECK(L.submit(make_job(descs[i]), ex.capacity(), nullptr, &id) == GRASP_OK);
        ids[i] = id;
        submitted.fetch_add(1);
        std::this_thread::sleep_for(std::chrono::microseconds(300 * (i % 4)));
      }
    });
  for (auto& t : th) t.join();
  th.clear();
  CHECK(submitted.load() == n_jobs);
  std::thread canceller([&] {
    for (int i = 0; i < n_jobs; ++i)
      if (want_cancel[i]) {
        // EINVAL when a poller already collected the (short) job
        const grasp_status c = L.cancel(ids[i]);
        CHECK(c == GRASP_OK || c == GRASP_EINVAL);
      }
  });
  std::vector<Result> res(n_jobs);
  for (int w = 0; w < 2; ++w)
    th.emplace_back([&, w] {
      for (int i = w; i < n_jobs; i += 2) res[i] = wait(L, ids[i], descs[i].B, descs[i].T);
    });
  canceller.join();
  for (auto& t : th) t.join();
  int done = 0, cancelled = 0;
  for (int i = 0; i < n_jobs; ++i) {
    const Result& r = res[i];
    CHECK(r.st == GRASP_OK || (want_cancel[i] && r.st == GRASP_ECANCELED));
    if (r.st == GRASP_ECANCELED) {
      ++cancelled;
      CHECK(r.steps <= descs[i].T);
      continue;
    }
    ++done;
    CHECK(r.steps == descs[i].T);
    std::vector<float> hist;
    const std::vector<float> alone = run_alone(descs[i], q0[i], &hist);
    CHECK(std::memcmp(alone.data(), r.q.data(), alone.size() * 4) == 0);
    if (descs[i].record_history) CHECK(std::memcmp(hist.data(), r.hist_loss.data(), hist.size() * 4) == 0);
    // ranking: a permutation in ascending loss order
    std::vector<int> seen(descs[i].B, 0);
    for (int k = 0; k < descs[i].B; ++k) {
      CHECK(r.rank[k] >= 0 && r.rank[k] < descs[i].B);
      seen[r.rank[k]]++;
      if (k) CHECK(r.loss[r.rank[k - 1]] <= r.loss[r.rank[k]]);
    }
    for (int s : seen) CHECK(s == 1);
    // a second poll forgets the job
    grasp_job_result again{};
    CHECK(L.poll(ids[i], &again) == GRASP_EINVAL);
    CHECK(L.cancel(ids[i]) == GRASP_EINVAL);
  }
  CHECK(ex.max_resident() <= 8);
  CHECK(ex.released() == n_jobs);
  grasp_serve_stats s{};
  L.stats(&s);
  CHECK(s.finished == n_jobs && s.queued == 0 && s.resident == 0);
  std::printf("mix: %d done, %d cancelled, %d steps, at most %d resident\n", done, cancelled, ex.steps(),
              ex.max_resident());
}

void test_full_arena_waits() {
  // room for one 16-candidate job at a time
  CpuExecutor ex(footprint_of(16) + 512);
  ServeLoop L(&ex, now);
  std::vector<std::vector<float>> q0(3);
  uint64_t ids[3];
  grasp_job_desc d[3];
  for (int i = 0; i < 3; ++i) {
    d[i] = make_desc(16, 4, 7 + i, q0[i]);
    CHECK(L.submit(make_job(d[i]), ex.capacity(), nullptr, &ids[i]) == GRASP_OK);
  }
  // a job larger than the arena can never fit
  std::vector<float> qb;
  uint64_t big = 0;
  CHECK(L.submit(make_job(make_desc(64, 2, 1, qb)), ex.capacity(), nullptr, &big) == GRASP_ENOMEM);
  Result r[3];
  for (int i = 0; i < 3; ++i) r[i] = wait(L, ids[i], 16, 4);
  for (int i = 0; i < 3; ++i) {
    CHECK(r[i].st == GRASP_OK && r[i].steps == 4);
    CHECK(std::memcmp(run_alone(d[i], q0[i], nullptr).data(), r[i].q.data(), r[i].q.size() * 4) == 0);
  }
  // one at a time, in arrival order: each admitted after the previous ended
  CHECK(ex.max_resident() == 1);
  CHECK(r[1].t_admit >= r[0].t_done && r[2].t_admit >= r[1].t_done);
  std::printf("full arena: jobs ran one after another\n");
}

void test_capacity_and_job_limit() {
  CpuExecutor ex(1 << 20);
  ServeLoop L(&ex, now);
  CHECK(L.configure(10, 2) == GRASP_OK);
  std::vector<float> q;
  uint64_t id;
  CHECK(L.submit(make_job(make_desc(11, 2, 3, q)), ex.capacity(), nullptr, &id) == GRASP_ENOMEM);
  std::vector<std::vector<float>> q0(6);
  std::vector<uint64_t> ids;
  for (int i = 0; i < 6; ++i) {
    CHECK(L.submit(make_job(make_desc(4, 3, 20 + i, q0[i])), ex.capacity(), nullptr, &id) == GRASP_OK);
    ids.push_back(id);
  }
  CHECK(L.configure(20, 2) == GRASP_EBUSY);
  for (uint64_t i : ids) CHECK(wait(L, i, 4, 3).st == GRASP_OK);
  // 4 + 4 candidates fit the capacity of 10, a third job would not; the job limit is 2 as well
  CHECK(ex.max_resident() == 2);
  std::printf("capacity and job limit held\n");
}

void test_executor_that_throws() {
  CpuExecutor ex(1 << 20, /*throw_at_step=*/3);
  ServeLoop L(&ex, now);
  std::vector<std::vector<float>> q0(4);
  std::vector<uint64_t> ids;
  for (int i = 0; i < 4; ++i) {
    uint64_t id;
    CHECK(L.submit(make_job(make_desc(3, 50, 40 + i, q0[i])), ex.capacity(), nullptr, &id) == GRASP_OK);
    ids.push_back(id);
  }
  for (uint64_t i : ids) {
    const Result r = wait(L, i, 3, 50);
    CHECK(r.st == GRASP_EDEVICE);
    CHECK(r.steps <= 3);
  }
  std::vector<float> q;
  uint64_t id;
  CHECK(L.submit(make_job(make_desc(3, 2, 1, q)), ex.capacity(), nullptr, &id) == GRASP_EDEVICE);
  CHECK(ex.released() == 4);
  std::printf("executor failure ended every job\n");
}

void test_shutdown_with_jobs_in_flight() {
  CpuExecutor ex(1 << 20);
  std::vector<std::vector<float>> q0(5);
  {
    ServeLoop L(&ex, now);
    CHECK(L.configure(64, 2) == GRASP_OK);
    for (int i = 0; i < 5; ++i) {
      uint64_t id;
      CHECK(L.submit(make_job(make_desc(2, 1000, 60 + i, q0[i])), ex.capacity(), nullptr, &id) == GRASP_OK);
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(20));
    L.shutdown();
    std::vector<float> q;
    uint64_t id;
    CHECK(L.submit(make_job(make_desc(2, 2, 1, q)), ex.capacity(), nullptr, &id) == GRASP_EINVAL);
  }
  CHECK(ex.released() == 5);
  std::printf("shutdown ended every job\n");
}

}  // namespace

int main() {
  test_mix_equals_alone();
  test_full_arena_waits();
  test_capacity_and_job_limit();
  test_executor_that_throws();
  test_shutdown_with_jobs_in_flight();
  std::printf("sched ok\n");
  return 0;
}
