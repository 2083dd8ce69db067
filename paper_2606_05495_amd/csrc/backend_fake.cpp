// CPU stand-in backend for scheduler tests: each worker "stream" is a thread
// that runs launched jobs in order, and completions are delivered on a
// separate callback thread (as a driver would).  It computes no pipeline; it
// writes the output header a device run would write, and it detects two jobs
// using one slot at the same time (the memory-safety invariant).
//
// Simulated job duration: vector jobs take n microseconds (n mod 10^6), all
// other pipelines take 20 microseconds.
#include <algorithm>
#include <cstdlib>
#include <condition_variable>
#include <deque>
#include <random>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace setrt {

namespace {

struct Pending {
  JobRec* job;
  DoneFn done;
  void* ctx;
};

class FakeBackend : public Backend {
 public:
  ~FakeBackend() override { shutdown(); }

  int init(const set_config& cfg, std::string*) override {
    cfg_ = cfg;
    b_ = cfg.num_workers;
    d_ = cfg.slots_per_worker;
    templates_.reserve(kMaxTemplates);  // entries never move while jobs read them
    inuse_.reserve(kMaxTemplates);
    workers_.resize(b_);
    for (int w = 0; w < b_; ++w) {
      workers_[w].reset(new Worker());
      workers_[w]->th = std::thread([this, w] { worker_loop(w); });
    }
    cb_thread_ = std::thread([this] { callback_loop(); });
    return SET_OK;
  }

  int define_template(int id, const set_job_template& t, std::string*) override {
    if ((int)templates_.size() != id) return SET_EINVAL;
    templates_.push_back(t);
    std::unique_ptr<std::atomic<int>[]> inuse(new std::atomic<int>[(size_t)b_ * d_]);
    for (int i = 0; i < b_ * d_; ++i) inuse[i] = 0;
    inuse_.push_back(std::move(inuse));
    return SET_OK;
  }

  int bind(JobRec* job, std::string*) override {
    // a real bind rewrites graph nodes of the slot's executable; that
    // executable must not be in flight (the slot is FREE when bound)
    if (inuse_[job->tmpl][(size_t)job->worker * d_ + job->slot].load()) violations_++;
    return SET_OK;
  }

  int launch(JobRec* job, DoneFn done, void* ctx, std::string* err) override {
    const int n = ++launches_;
    if (cfg_.fake_fail_after > 0 && n >= cfg_.fake_fail_after) {
      if (err) *err = "injected launch failure";
      return SET_EDEVICE;
    }
    Worker& w = *workers_[job->worker];
    {
      std::lock_guard<std::mutex> g(w.mu);
      w.q.push_back(Pending{job, done, ctx});
    }
    w.cv.notify_one();
    return SET_OK;
  }

  int launch_polled(JobRec* job, std::string* err) override {
    const int n = ++launches_;
    if (cfg_.fake_fail_after > 0 && n >= cfg_.fake_fail_after) {
      if (err) *err = "injected launch failure";
      return SET_EDEVICE;
    }
    {
      std::lock_guard<std::mutex> g(done_mu_);
      done_[job] = false;
    }
    Worker& w = *workers_[job->worker];
    {
      std::lock_guard<std::mutex> g(w.mu);
      w.q.push_back(Pending{job, nullptr, nullptr});
    }
    w.cv.notify_one();
    return SET_OK;
  }
  int is_done(JobRec* job, bool* done, std::string*) override {
    std::lock_guard<std::mutex> g(done_mu_);
    auto it = done_.find(job);
    *done = (it != done_.end() && it->second);
    if (*done) done_.erase(it);
    return SET_OK;
  }

  int run_sync(JobRec* job, int, std::string*) override {
    execute(job);
    return SET_OK;
  }
  int run_graph(JobRec* job, int, std::string*) override {
    execute(job);
    return SET_OK;
  }
  int run_batch(JobRec** jobs, int count, std::string*) override {
    uint64_t longest = 0;
    for (int i = 0; i < count; ++i) longest = std::max(longest, duration_us(jobs[i]));
    sleep_us(longest);
    for (int i = 0; i < count; ++i) write_header(jobs[i], true);
    return SET_OK;
  }
  void* alloc_host(uint64_t bytes) override { return std::calloc(1, bytes); }
  void free_host(void* p) override { std::free(p); }
  int time_stage(int, int, int, int, double* avg_us, std::string*) override {
    *avg_us = 0.0;
    return SET_OK;
  }
  int time_device_copy(uint64_t, int, double*, std::string* err) override {
    if (err) *err = "the fake backend has no device";
    return SET_EUNSUPPORTED;
  }

  void shutdown() override {
    if (stop_.exchange(true)) return;
    for (auto& w : workers_) {
      {
        std::lock_guard<std::mutex> g(w->mu);
        w->cv.notify_all();
      }
      if (w->th.joinable()) w->th.join();
    }
    {
      std::lock_guard<std::mutex> g(cb_mu_);
      cb_cv_.notify_all();
    }
    if (cb_thread_.joinable()) cb_thread_.join();
  }

 private:
  struct Worker {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Pending> q;
    std::thread th;
  };

  // A job's simulated run time, plus the template's stress delay.
  uint64_t duration_us(const JobRec* j) const {
    const set_job_template& t = templates_[j->tmpl];
    if (t.pipeline == SET_PIPE_SAXPY_TANH_SUM_F32) return j->args.n % 1000000ull + t.stress_delay_us;
    return 20 + t.stress_delay_us;
  }
  static void sleep_us(uint64_t us) {
    if (us) std::this_thread::sleep_for(std::chrono::microseconds(us));
  }

  void write_header(JobRec* j, bool ok) {
    if (!j->args.host_out || j->args.out_bytes < sizeof(set_out_header)) return;
    set_out_header h{};
    h.job_id = j->id;
    h.seq = j->seq;
    h.worker = (uint32_t)j->worker;
    h.slot = (uint32_t)j->slot;
    h.magic = SET_OUT_MAGIC;
    h.canary_ok = ok ? 1u : 0u;
    h.user_tag = j->args.user_tag;
    std::memcpy(j->args.host_out, &h, sizeof(h));
  }

  // Runs one job on the calling thread; returns false if its slot was busy.
  bool execute(JobRec* j) {
    std::atomic<int>& u = inuse_[j->tmpl][(size_t)j->worker * d_ + j->slot];
    const bool clash = u.exchange(1) != 0;
    if (clash) violations_++;
    sleep_us(duration_us(j));
    write_header(j, !clash && violations_.load() == 0);
    u.store(0);
    return !clash;
  }

  void worker_loop(int wi) {
    Worker& w = *workers_[wi];
    while (true) {
      Pending p;
      {
        std::unique_lock<std::mutex> lk(w.mu);
        w.cv.wait(lk, [&] { return stop_.load() || !w.q.empty(); });
        if (w.q.empty()) return;
        p = w.q.front();
        w.q.pop_front();
      }
      execute(p.job);
      if (!p.done) {  // queue model: completion is observed by polling
        std::lock_guard<std::mutex> g(done_mu_);
        done_[p.job] = true;
        continue;
      }
      {
        std::lock_guard<std::mutex> g(cb_mu_);
        cb_q_.push_back(p);
      }
      cb_cv_.notify_one();
    }
  }

  void callback_loop() {
    std::mt19937 rng(12345);
    while (true) {
      std::vector<Pending> batch;
      {
        std::unique_lock<std::mutex> lk(cb_mu_);
        cb_cv_.wait(lk, [&] { return stop_.load() || !cb_q_.empty(); });
        if (cb_q_.empty()) return;
        batch.assign(cb_q_.begin(), cb_q_.end());
        cb_q_.clear();
      }
      if (cfg_.fake_reorder_callbacks) std::shuffle(batch.begin(), batch.end(), rng);
      for (auto& p : batch) p.done(p.ctx, p.job, SET_OK);
    }
  }

  set_config cfg_{};
  int b_ = 0, d_ = 0;
  std::vector<set_job_template> templates_;
  std::vector<std::unique_ptr<std::atomic<int>[]>> inuse_;
  std::vector<std::unique_ptr<Worker>> workers_;
  std::mutex cb_mu_;
  std::condition_variable cb_cv_;
  std::deque<Pending> cb_q_;
  std::thread cb_thread_;
  std::atomic<bool> stop_{false};
  std::atomic<int> launches_{0};
  std::atomic<int> violations_{0};
  std::mutex done_mu_;
  std::unordered_map<JobRec*, bool> done_;
};

}  // namespace

Backend* make_fake_backend() { return new FakeBackend(); }

}  // namespace setrt

#ifdef SET_NO_HIP_BACKEND
// Host-only builds (the ThreadSanitizer driver) carry no device code.
namespace setrt {
Backend* make_hip_backend() { return nullptr; }
}  // namespace setrt
#endif
