// Scheduler core and C ABI.  Backend-agnostic: the same code drives the HIP
// backend and the CPU fake backend.
//
// SET mode follows Section 4.2:
//  * workers W_i = stream + per-slot graph executables + slot buffers;
//  * per-worker bounded queues Q_i of fully bound jobs (Section 4.2 (2));
//  * a free-worker pool W_pool holding launch permits, refilled only by
//    completions (Section 4.2 (3));
//  * a submitter thread (Algorithm 1) and a dispatcher thread (Algorithm 2:
//    FindJob = local pop, else steal from (w+k) mod b; LaunchJob = retarget if
//    stolen, launch, add the completion callback);
//  * completion (Algorithm 3): c_done += 1, permit back to W_pool, notify.
// Readings of points the paper leaves open:
//  * one executable per (worker, slot) and up to d slots per worker, so a
//    queue holds several prepared executables of its worker;
//  * W_pool holds per-worker launch permits (in-flight depth k per worker);
//  * a dispatcher whose token finds no job returns it to the pool and sleeps
//    until the submitter pushes or a completion arrives (no polling);
//  * a thief takes the oldest job of a victim queue;
//  * job ids are claimed at set_submit time in submission order.
#include <algorithm>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <memory>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace setrt {

namespace {

thread_local std::string g_create_error;

// Timed condition wait on the system clock (pthread_cond_timedwait); the
// steady-clock form is not observed by thread sanitizers on this toolchain.
template <class Pred>
bool timed_wait(std::condition_variable& cv, std::unique_lock<std::mutex>& lk, std::chrono::nanoseconds d,
                Pred pred) {
  return cv.wait_until(lk, std::chrono::system_clock::now() + d, pred);
}

// Bounded FIFO of bound jobs for one worker (Q_i).  The owner pops the head;
// a thief takes the head as well.
class WorkerQueue {
 public:
  void init(int cap) {
    cap_ = cap;
    ring_.assign(cap, nullptr);
  }
  bool try_push(JobRec* j, uint32_t* size_after) {
    std::lock_guard<std::mutex> g(mu_);
    if (count_ >= cap_) return false;
    ring_[(head_ + count_) % cap_] = j;
    ++count_;
    if (size_after) *size_after = (uint32_t)count_;
    return true;
  }
  JobRec* try_pop() {
    std::lock_guard<std::mutex> g(mu_);
    if (count_ == 0) return nullptr;
    JobRec* j = ring_[head_];
    head_ = (head_ + 1) % cap_;
    --count_;
    return j;
  }
  // Steal the head only if accept(job) agrees (the thief has a free slot).
  template <class F>
  JobRec* try_steal_if(F accept) {
    std::lock_guard<std::mutex> g(mu_);
    if (count_ == 0) return nullptr;
    JobRec* j = ring_[head_];
    if (!accept(j)) return nullptr;
    head_ = (head_ + 1) % cap_;
    --count_;
    return j;
  }
  int size() {
    std::lock_guard<std::mutex> g(mu_);
    return count_;
  }
  bool full() {
    std::lock_guard<std::mutex> g(mu_);
    return count_ >= cap_;
  }

 private:
  std::mutex mu_;
  std::vector<JobRec*> ring_;
  int cap_ = 0, head_ = 0, count_ = 0;
};

}  // namespace

void set_thread_error(const std::string& msg) { g_create_error = msg; }

class Context {
 public:
  set_config cfg{};
  std::unique_ptr<Backend> be;
  int b = 0, d = 0, qcap = 0, kperm = 0;

  // ---- error latch
  std::mutex err_mu;
  std::string last_error;
  std::atomic<int> sticky{SET_OK};

  // ---- templates
  // Capacity kMaxTemplates is reserved up front, so a template defined while
  // jobs of others run never moves the entries those jobs read; ntmpl
  // publishes a new entry once it is complete.
  std::vector<set_job_template> templates;
  std::vector<TemplateSizes> tsizes;
  // free-slot bitmask per (template, worker): bit s set = slot FREE
  std::vector<std::unique_ptr<std::atomic<uint64_t>[]>> free_mask;
  // [tmpl][w*d+s]: touched only by the thread that holds the slot (binder, or a thief retargeting to its own slot)
  std::vector<std::vector<uint64_t>> slot_seq;
  std::atomic<int> ntmpl{0};
  bool valid_template(int id) const { return id >= 0 && id < ntmpl.load(std::memory_order_acquire); }

  // ---- job records
  std::mutex job_mu;
  std::vector<std::unique_ptr<JobRec[]>> job_chunks;
  JobRec* job_free = nullptr;

  // ---- staging (set_submit -> submitter)
  std::mutex stage_mu;
  std::condition_variable stage_cv;       // submitter waits for jobs
  std::condition_variable stage_room_cv;  // producers wait for room
  std::deque<JobRec*> staging;
  int staging_cap = 4096;

  // ---- SET structures
  std::vector<std::unique_ptr<WorkerQueue>> queues;
  // W_pool, split by dispatcher thread: dispatcher t holds the launch
  // permits of workers w with w % ndisp == t, so each worker's launches come
  // from one thread and keep their order on its stream.
  struct DispState {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<int> pool;              // launch permits (worker ids)
    std::atomic<uint64_t> pool_gen{0};
  };
  int ndisp = 1;
  std::vector<std::unique_ptr<DispState>> disp;
  std::atomic<int64_t> queued{0};  // jobs sitting in any Q_i
  std::atomic<uint64_t> push_gen{0};
  std::mutex sub_mu;
  std::condition_variable sub_cv;  // submitter waits for queue room / slots / budget
  std::atomic<uint64_t> room_gen{0};
  int rr_next = 0;

  std::atomic<uint64_t> c_next{0};  // next job id
  std::atomic<uint64_t> c_done{0};  // completed jobs
  std::mutex done_mu;
  std::condition_variable done_cv;

  std::thread submitter;
  std::vector<std::thread> dispatchers;
  std::atomic<bool> stopping{false};

  // ---- queue model (SET_MODE_QUEUE)
  std::mutex gq_mu;            // the global issue-queue mutex
  std::deque<JobRec*> gq;
  std::thread issuer;

  // ---- baseline modes
  std::mutex base_mu;
  std::vector<JobRec*> batch;
  uint64_t rr_stream = 0;

  // ---- stats
  std::atomic<uint64_t> st_completed{0}, st_stolen{0}, st_failed{0};
  std::atomic<uint64_t> st_launch[kMaxWorkers];
  std::atomic<int> free_permits[kMaxWorkers];  // launch permits of each worker sitting in a pool
  std::atomic<uint64_t> st_ns_bind{0}, st_ns_launch{0}, st_ns_cb{0}, st_ns_sync{0};
  std::atomic<uint32_t> st_q_hw{0}, st_inflight_hw{0};
  std::atomic<int64_t> inflight{0};
  std::atomic<uint64_t> st_h2d{0}, st_d2h{0};
  std::atomic<uint64_t> mem_in_use{0}, st_mem_hw{0};
  std::atomic<uint64_t> st_batches{0};
  std::atomic<uint64_t> t_first_submit{0}, t_last_done{0};
  std::atomic<uint64_t> submitted_base{0};  // c_next at last reset
  std::mutex times_mu;
  std::vector<set_job_times> times;

  std::atomic<set_completion_fn> user_fn{nullptr};
  std::atomic<void*> user_arg{nullptr};

  // ---- serving (set_serve)
  struct VecRing {
    char* tab = nullptr;
    char* res = nullptr;
    std::vector<uint32_t> idx;
    bool busy = false;
  };
  struct ServeState {
    const set_request* reqs = nullptr;
    uint64_t* done_ns = nullptr;
    float* vec_results = nullptr;
    uint64_t t0 = 0;
    int vtmpl = -1;
    uint32_t vec_batch_max = 0, vec_inflight_max = 0;
    const set_vec_tuning* tuning = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint32_t> pending;
    std::vector<VecRing> ring;
    uint32_t inflight = 0;
    bool arrivals_done = false;
    std::atomic<uint64_t> completed{0}, failed{0}, batches{0}, t_last{0};
  };
  ServeState* serve_st = nullptr;

  // ---- set_run_vector_jobs: pinned staging of descriptor tables and results
  // (grow-only, freed at shutdown); the mutex serialises concurrent calls
  std::mutex vec_stage_mu;
  char* vec_stage = nullptr;
  uint64_t vec_stage_bytes = 0;

  ~Context() { shutdown(); }

  // ------------------------------------------------------------------ errors
  int fail(int code, const std::string& msg) {
    {
      std::lock_guard<std::mutex> g(err_mu);
      last_error = msg;
    }
    if (code == SET_EDEVICE) {
      int expect = SET_OK;
      sticky.compare_exchange_strong(expect, SET_EDEVICE);
    }
    return code;
  }
  int check_sticky() { return sticky.load(std::memory_order_acquire); }

  // ------------------------------------------------------------------ job records
  JobRec* alloc_job() {
    std::lock_guard<std::mutex> g(job_mu);
    if (!job_free) {
      const int n = 1024;
      std::unique_ptr<JobRec[]> chunk(new JobRec[n]);
      for (int i = 0; i < n; ++i) {
        chunk[i].next = job_free;
        job_free = &chunk[i];
      }
      job_chunks.push_back(std::move(chunk));
    }
    JobRec* j = job_free;
    job_free = j->next;
    std::memset(j, 0, sizeof(*j));
    j->serve_ref = -1;
    return j;
  }
  void free_job(JobRec* j) {
    std::lock_guard<std::mutex> g(job_mu);
    j->next = job_free;
    job_free = j;
  }

  // ------------------------------------------------------------------ slots
  int acquire_slot(int tmpl, int w) {
    std::atomic<uint64_t>& m = free_mask[tmpl][w];
    uint64_t cur = m.load(std::memory_order_acquire);
    while (cur) {
      const int s = __builtin_ctzll(cur);
      if (m.compare_exchange_weak(cur, cur & ~(1ull << s), std::memory_order_acq_rel)) return s;
    }
    return -1;
  }
  void release_slot(int tmpl, int w, int s) { free_mask[tmpl][w].fetch_or(1ull << s, std::memory_order_acq_rel); }

  bool budget_allows(uint64_t fp) {
    if (cfg.mem_budget_bytes == 0) return true;
    uint64_t cur = mem_in_use.load();
    while (cur + fp <= cfg.mem_budget_bytes) {
      if (mem_in_use.compare_exchange_weak(cur, cur + fp)) {
        update_max(st_mem_hw, cur + fp);
        return true;
      }
    }
    return false;
  }
  template <class A, class V>
  static void update_max(A& a, V v) {
    auto cur = a.load();
    while (v > cur && !a.compare_exchange_weak(cur, v)) {
    }
  }

  // Bind job j to (w, s): UpdateGraphParams (Algorithm 1; Algorithm 2 on a steal).
  int bind_to(JobRec* j, int w, int s) {
    j->worker = w;
    j->slot = s;
    j->seq = ++slot_seq[j->tmpl][(size_t)w * d + s];
    const uint64_t t0 = now_ns();
    std::string err;
    int rc = be->bind(j, &err);
    st_ns_bind += now_ns() - t0;
    if (rc != SET_OK) return fail(rc, "bind: " + err);
    return SET_OK;
  }

  // ------------------------------------------------------------------ init
  int init(const set_config& c) {
    cfg = c;
    b = c.num_workers;
    d = c.slots_per_worker;
    kperm = c.inflight_per_worker > 0 ? c.inflight_per_worker : std::min(2, d);
    qcap = c.queue_capacity > 0 ? c.queue_capacity : std::max(1, d - kperm);
    staging_cap = c.staging_capacity > 0 ? c.staging_capacity : 4096;
    templates.reserve(kMaxTemplates);
    tsizes.reserve(kMaxTemplates);
    free_mask.reserve(kMaxTemplates);
    slot_seq.reserve(kMaxTemplates);
    for (int i = 0; i < kMaxWorkers; ++i) {
      st_launch[i] = 0;
      free_permits[i] = 0;
    }
    // A thief steals only into a FREE slot of its own; with an empty queue and a
    // permit in hand it has at most kperm - 1 slots in flight, so kperm <= d
    // guarantees progress (q + k <= d additionally guarantees every steal finds a slot).
    if (c.mode == SET_MODE_SET && kperm > d)
      return fail(SET_EINVAL, "inflight_per_worker must not exceed slots_per_worker");
    be.reset(c.backend == SET_BACKEND_FAKE ? make_fake_backend() : make_hip_backend());
    if (!be) return fail(SET_EUNSUPPORTED, "backend not available in this build");
    std::string err;
    int rc = be->init(cfg, &err);
    if (rc != SET_OK) return fail(rc, "backend init: " + err);
    if (cfg.mode == SET_MODE_SET) {
      queues.resize(b);
      for (int i = 0; i < b; ++i) {
        queues[i].reset(new WorkerQueue());
        queues[i]->init(qcap);
      }
      ndisp = std::max(1, std::min(cfg.dispatch_threads, b));
      for (int t = 0; t < ndisp; ++t) disp.emplace_back(new DispState());
      // permits interleaved across workers so the first launches spread out
      for (int r = 0; r < kperm; ++r)
        for (int w = 0; w < b; ++w) disp[w % ndisp]->pool.push_back(w);
      for (int w = 0; w < b; ++w) free_permits[w] = kperm;
      submitter = std::thread([this] { submitter_loop(); });
      for (int t = 0; t < ndisp; ++t) dispatchers.emplace_back([this, t] { dispatcher_loop(t); });
    }
    if (cfg.mode == SET_MODE_QUEUE) issuer = std::thread([this] { issuer_loop(); });
    return SET_OK;
  }

  void shutdown() {
    if (!stopping.exchange(true)) {
      {
        std::lock_guard<std::mutex> g(stage_mu);
        stage_cv.notify_all();
        stage_room_cv.notify_all();
      }
      for (auto& ds : disp) {
        std::lock_guard<std::mutex> g(ds->mu);
        ds->cv.notify_all();
      }
      {
        std::lock_guard<std::mutex> g(sub_mu);
        sub_cv.notify_all();
      }
      if (submitter.joinable()) submitter.join();
      for (auto& th : dispatchers)
        if (th.joinable()) th.join();
      if (issuer.joinable()) issuer.join();
      if (be && vec_stage) be->free_host(vec_stage);
      vec_stage = nullptr;
      if (be) be->shutdown();
    }
  }

  int define_template(const set_job_template& t, int* id) {
    if (ntmpl.load() >= kMaxTemplates) return fail(SET_EINVAL, "too many templates");
    std::string why;
    if (pipeline_validate(t, &why) != SET_OK) return fail(SET_EINVAL, why);
    if (t.pipeline == SET_PIPE_SCAN_LIB_I32_I64 && cfg.mode == SET_MODE_BATCH_SYNC)
      return fail(SET_EUNSUPPORTED, "library-call templates are captured per slot; no batch graph is built for them");
    TemplateSizes sz;
    pipeline_sizes(t, &sz);
    const int tid = (int)templates.size();
    std::string err;
    int rc = be->define_template(tid, t, &err);
    if (rc != SET_OK) return fail(rc, "define_template: " + err);
    std::unique_ptr<std::atomic<uint64_t>[]> masks(new std::atomic<uint64_t>[b]);
    const uint64_t all = (d >= 64) ? ~0ull : ((1ull << d) - 1);
    for (int w = 0; w < b; ++w) masks[w] = all;
    free_mask.push_back(std::move(masks));
    slot_seq.emplace_back((size_t)b * d, 0);
    tsizes.push_back(sz);
    templates.push_back(t);
    ntmpl.store(tid + 1, std::memory_order_release);
    *id = tid;
    return SET_OK;
  }

  // ------------------------------------------------------------------ completion (Algorithm 3)
  static void on_done_tramp(void* ctx, JobRec* j, int status) { static_cast<Context*>(ctx)->on_done(j, status); }

  void record_done(JobRec* j, int status) {
    j->t_done = now_ns();
    j->status = status;
    if (status != SET_OK) ++st_failed;
    ++st_completed;
    const set_job_args& a = j->args;
    st_h2d += a.in_bytes;
    st_d2h += pipeline_out_bytes(templates[j->tmpl], a.n);
    update_max(t_last_done, j->t_done);
    {
      std::lock_guard<std::mutex> g(times_mu);
      if (times.size() < (1u << 22))
        times.push_back(set_job_times{j->id, j->t_submit, j->t_launch, j->t_done, j->worker, j->slot, j->stolen,
                                      status});
    }
    if (j->serve_ref != -1 && serve_st) serve_complete(j, status);
    set_completion_fn fn = user_fn.load();
    if (fn) fn(j->id, status, user_arg.load());
  }

  void serve_complete(JobRec* j, int status) {
    ServeState& S = *serve_st;
    const uint64_t now = now_ns() - S.t0;
    update_max(S.t_last, now);
    if (j->serve_ref >= 0) {
      if (status == SET_OK) {
        S.done_ns[j->serve_ref] = now;
        ++S.completed;
      } else {
        ++S.failed;
      }
      return;
    }
    const int r = (int)(-2 - j->serve_ref);
    VecRing& R = S.ring[r];
    const set_out_header* h = reinterpret_cast<const set_out_header*>(R.res);
    const bool ok = status == SET_OK && h->magic == SET_OUT_MAGIC && h->canary_ok == 1;
    if (ok) {
      const float* v = reinterpret_cast<const float*>(R.res + 64);
      for (size_t q = 0; q < R.idx.size(); ++q) {
        if (S.vec_results) S.vec_results[R.idx[q]] = v[q];
        S.done_ns[R.idx[q]] = now;
      }
      S.completed += R.idx.size();
    } else {
      S.failed += R.idx.size();
    }
    {
      std::lock_guard<std::mutex> g(S.mu);
      R.busy = false;
      R.idx.clear();
      --S.inflight;
    }
    S.cv.notify_all();
  }

  void on_done(JobRec* j, int status) {
    const uint64_t t0 = now_ns();
    const int w = j->worker, s = j->slot, tmpl = j->tmpl;
    const uint64_t fp = j->footprint;
    record_done(j, status);
    release_slot(tmpl, w, s);
    if (cfg.mem_budget_bytes) mem_in_use -= fp;
    --inflight;
    free_job(j);
    {
      DispState& ds = *disp[w % ndisp];
      {
        std::lock_guard<std::mutex> g(ds.mu);
        ds.pool.push_back(w);  // W_pool.push(w)
        ++free_permits[w];
        ++ds.pool_gen;
      }
      ds.cv.notify_one();  // notify_one()
    }
    {
      std::lock_guard<std::mutex> g(sub_mu);
      ++room_gen;
    }
    sub_cv.notify_one();
    {
      std::lock_guard<std::mutex> g(done_mu);
      c_done.fetch_add(1);  // c_done.atomic_fetch_add(1)
    }
    done_cv.notify_all();
    st_ns_cb += now_ns() - t0;
  }

  // ------------------------------------------------------------------ submitter (Algorithm 1)
  int pick_worker(JobRec* j, int* slot_out) {
    const int tmpl = j->tmpl;
    auto try_w = [&](int w) -> bool {
      if (queues[w]->full()) return false;
      int s = acquire_slot(tmpl, w);
      if (s < 0) return false;
      *slot_out = s;
      return true;
    };
    if (j->args.worker_hint >= 0) return try_w(j->args.worker_hint % b) ? j->args.worker_hint % b : -1;
    if (cfg.submit_policy == SET_SUBMIT_SKEW0) return try_w(0) ? 0 : -1;
    if (cfg.submit_policy == SET_SUBMIT_SHORTEST) {
      int best = -1, best_sz = 1 << 30;
      for (int k = 0; k < b; ++k) {
        const int sz = queues[k]->size();
        if (sz < best_sz && !queues[k]->full() && free_mask[tmpl][k].load() != 0) {
          best = k;
          best_sz = sz;
        }
      }
      if (best >= 0 && try_w(best)) return best;
      return -1;
    }
    for (int k = 0; k < b; ++k) {
      const int w = (rr_next + k) % b;
      if (try_w(w)) {
        rr_next = (w + 1) % b;
        return w;
      }
    }
    return -1;
  }

  // Admission (Algorithm 1): scan up to kAdmitWindow staged jobs in order.  A
  // job whose template has no free slot on a worker with queue room is
  // skipped together with every later job of that template (per-template
  // order is kept); the memory budget is strictly first-come first-served: a
  // job blocked by the budget is never overtaken, so large jobs cannot starve.
  // Returns 1 if a job was admitted, 0 if none could be, -1 on a bind error.
  static constexpr size_t kAdmitWindow = 32;

  int admit_one() {
    JobRec* window[kAdmitWindow];
    size_t nw = 0;
    {
      std::lock_guard<std::mutex> g(stage_mu);
      for (; nw < kAdmitWindow && nw < staging.size(); ++nw) window[nw] = staging[nw];
    }
    uint64_t blocked = 0;  // templates with no free slot this round
    for (size_t k = 0; k < nw; ++k) {
      JobRec* j = window[k];
      if (blocked & (1ull << j->tmpl)) continue;
      if (!budget_allows(j->footprint)) return 0;
      int s = -1;
      const int w = pick_worker(j, &s);
      if (w < 0) {
        if (cfg.mem_budget_bytes) mem_in_use -= j->footprint;
        blocked |= 1ull << j->tmpl;
        continue;
      }
      {
        std::lock_guard<std::mutex> g(stage_mu);
        staging.erase(std::find(staging.begin(), staging.begin() + (k + 1), j));
      }
      stage_room_cv.notify_all();
      if (bind_to(j, w, s) != SET_OK) {
        release_slot(j->tmpl, w, s);
        if (cfg.mem_budget_bytes) mem_in_use -= j->footprint;
        fail_unlaunched(j);
        return -1;
      }
      uint32_t sz = 0;
      queues[w]->try_push(j, &sz);  // cannot fail: only this thread pushes and pick_worker saw room
      update_max(st_q_hw, sz);
      ++queued;
      ++push_gen;
      wake_dispatchers(w);
      return 1;
    }
    return 0;
  }

  void submitter_loop() {
    while (true) {
      {
        std::unique_lock<std::mutex> lk(stage_mu);
        stage_cv.wait(lk, [&] { return stopping.load() || !staging.empty(); });
        if (staging.empty()) return;  // stopping and nothing left
      }
      if (check_sticky() != SET_OK) {
        // the context is latched into an error: staged jobs complete as failed
        JobRec* j = nullptr;
        {
          std::lock_guard<std::mutex> g(stage_mu);
          j = staging.front();
          staging.pop_front();
        }
        stage_room_cv.notify_all();
        fail_unlaunched(j);
        continue;
      }
      const uint64_t gen = room_gen.load();
      if (admit_one() != 0) continue;
      std::unique_lock<std::mutex> lk(sub_mu);
      timed_wait(sub_cv, lk, std::chrono::milliseconds(50), [&] { return room_gen.load() != gen || stopping.load(); });
    }
  }

  // A job that never reached the device completes with SET_EDEVICE.
  void fail_unlaunched(JobRec* j) {
    record_done(j, SET_EDEVICE);
    free_job(j);
    {
      std::lock_guard<std::mutex> g(done_mu);
      c_done.fetch_add(1);
    }
    done_cv.notify_all();
  }

  // ------------------------------------------------------------------ dispatcher (Algorithm 2)
  JobRec* find_job(int w) {
    JobRec* j = queues[w]->try_pop();
    if (j) {
      j->stolen = 0;
      return j;
    }
    if (!cfg.work_stealing) return nullptr;
    for (int k = 1; k < b; ++k) {
      const int v = (w + k) % b;
      // SET_STEAL_BUSY: a victim holding a free permit launches the job itself
      if (cfg.steal_policy == SET_STEAL_BUSY && free_permits[v].load(std::memory_order_relaxed) > 0) continue;
      int new_slot = -1;
      JobRec* s = queues[v]->try_steal_if([&](JobRec* cand) {
        new_slot = acquire_slot(cand->tmpl, w);
        return new_slot >= 0;
      });
      if (s) {
        // retarget to the thief's buffers; the victim's pre-bound slot returns FREE unused
        const int old_w = s->worker, old_s = s->slot;
        s->stolen = 1;
        if (bind_to(s, w, new_slot) != SET_OK) {
          // (w, new_slot) stays with the job and is released by its failed completion
          release_slot(s->tmpl, old_w, old_s);
          s->status = SET_EDEVICE;
          return s;
        }
        release_slot(s->tmpl, old_w, old_s);
        {
          std::lock_guard<std::mutex> g(sub_mu);
          ++room_gen;
        }
        sub_cv.notify_one();
        ++st_stolen;
        return s;
      }
    }
    return nullptr;
  }

  void launch_job(JobRec* j, int w) {
    {
      std::lock_guard<std::mutex> g(sub_mu);
      ++room_gen;  // queue room freed
    }
    sub_cv.notify_one();
    if (j->status != SET_OK || check_sticky() != SET_OK) {
      ++inflight;
      on_done(j, SET_EDEVICE);
      return;
    }
    j->t_launch = now_ns();
    const int64_t inf = ++inflight;
    update_max(st_inflight_hw, (uint32_t)inf);
    ++st_launch[w];
    std::string err;
    const uint64_t t0 = now_ns();
    int rc = be->launch(j, &Context::on_done_tramp, this, &err);
    st_ns_launch += now_ns() - t0;
    if (rc != SET_OK) {
      fail(rc, "launch: " + err);
      on_done(j, rc);
    }
  }

  // A job was pushed to Q_w: wake w's dispatcher, and with stealing the
  // others too (a thief with a free permit may take it).
  void wake_dispatchers(int w) {
    for (int t = 0; t < ndisp; ++t) {
      if (t != w % ndisp && !cfg.work_stealing) continue;
      DispState& ds = *disp[t];
      { std::lock_guard<std::mutex> g(ds.mu); }
      ds.cv.notify_one();
    }
  }

  void dispatcher_loop(int t) {
    DispState& ds = *disp[t];
    std::vector<int> snapshot;
    while (true) {
      uint64_t gen_seen, pool_seen;
      {
        std::unique_lock<std::mutex> lk(ds.mu);
        auto ready = [&] { return (!ds.pool.empty() && queued.load() > 0) || stopping.load(); };
        if (!ready() && cfg.spin_us > 0) {
          lk.unlock();
          const uint64_t until = now_ns() + (uint64_t)cfg.spin_us * 1000ull;
          while (now_ns() < until) {
            if (queued.load(std::memory_order_relaxed) > 0) break;
            std::this_thread::yield();
          }
          lk.lock();
        }
        ds.cv.wait(lk, ready);
        if (stopping.load() && queued.load() == 0) return;
        snapshot.assign(ds.pool.begin(), ds.pool.end());
        gen_seen = push_gen.load();
        pool_seen = ds.pool_gen.load();
      }
      // W_pool.pop(), FindJob; a permit that finds nothing goes back (reading 1).
      // Only this thread removes permits from its pool, so each snapshot
      // entry is still there when it is taken below.
      int chosen = -1;
      JobRec* job = nullptr;
      for (size_t i = 0; i < snapshot.size() && !job; ++i) {
        const int w = snapshot[i];
        bool tried = false;
        for (size_t k = 0; k < i; ++k) tried |= (snapshot[k] == w);
        if (tried) continue;
        job = find_job(w);
        if (job) chosen = w;
      }
      if (!job) {
        std::unique_lock<std::mutex> lk(ds.mu);
        timed_wait(ds.cv, lk, std::chrono::milliseconds(20), [&] {
          return push_gen.load() != gen_seen || ds.pool_gen.load() != pool_seen ||
                 (stopping.load() && queued.load() == 0);
        });
        continue;
      }
      {
        std::lock_guard<std::mutex> g(ds.mu);
        ds.pool.erase(std::find(ds.pool.begin(), ds.pool.end(), chosen));
        --free_permits[chosen];
      }
      --queued;
      launch_job(job, chosen);  // LaunchJob
    }
  }

  // ------------------------------------------------------------------ queue model (baseline)
  // The issuer holds the global mutex for a whole round in which it queries
  // every worker: finished jobs complete, idle workers get the next job.
  void complete_polled(JobRec* j, int status) {
    record_done(j, status);
    free_job(j);
    {
      std::lock_guard<std::mutex> g(done_mu);
      c_done.fetch_add(1);
    }
    done_cv.notify_all();
  }

  void issuer_loop() {
    std::vector<JobRec*> running(b, nullptr);
    while (true) {
      bool progressed = false, busy = false;
      {
        std::lock_guard<std::mutex> g(gq_mu);
        for (int w = 0; w < b; ++w) {
          std::string err;
          if (running[w]) {
            bool done = false;
            const int rc = be->is_done(running[w], &done, &err);
            if (rc != SET_OK) {
              fail(rc, "queue model: " + err);
              done = true;
            }
            if (done) {
              complete_polled(running[w], rc);
              running[w] = nullptr;
              progressed = true;
            }
          }
          if (!running[w] && !gq.empty()) {
            JobRec* j = gq.front();
            gq.pop_front();
            j->worker = w;
            j->slot = 0;
            j->seq = ++slot_seq[j->tmpl][(size_t)w * d];
            int rc = check_sticky();
            if (rc == SET_OK) {
              const uint64_t t0 = now_ns();
              rc = be->bind(j, &err);
              st_ns_bind += now_ns() - t0;
            }
            if (rc == SET_OK) {
              j->t_launch = now_ns();
              ++st_launch[w];
              const uint64_t t1 = now_ns();
              rc = be->launch_polled(j, &err);
              st_ns_launch += now_ns() - t1;
            }
            if (rc != SET_OK) {
              if (rc != check_sticky()) fail(rc, "queue model: " + err);
              complete_polled(j, SET_EDEVICE);
            } else {
              running[w] = j;
            }
            progressed = true;
          }
          busy |= running[w] != nullptr;
        }
        if (!busy && gq.empty() && stopping.load()) return;
      }
      if (!progressed) std::this_thread::yield();
    }
  }

  // ------------------------------------------------------------------ submit
  int submit(int tmpl, const set_job_args* a, int flags, uint64_t* id_out, int64_t serve_ref = -1) {
    int st = check_sticky();
    if (st != SET_OK) return st;
    if (stopping.load()) return SET_ECLOSED;
    if (!valid_template(tmpl)) return fail(SET_EINVAL, "unknown template id");
    if (!a) return fail(SET_EINVAL, "null job args");
    std::string why;
    if (pipeline_validate_job(templates[tmpl], *a, &why) != SET_OK) return fail(SET_EINVAL, why);
    if (cfg.mem_budget_bytes && tsizes[tmpl].slot_bytes > cfg.mem_budget_bytes)
      return fail(SET_EINVAL, "the template's slot footprint exceeds the memory budget");
    JobRec* j = alloc_job();
    j->tmpl = tmpl;
    j->args = *a;
    j->serve_ref = serve_ref;
    if ((templates[tmpl].pipeline == SET_PIPE_SCAN_I32_I64 || templates[tmpl].pipeline == SET_PIPE_SCAN_LIB_I32_I64) &&
        j->args.n == 0)
      j->args.n = templates[tmpl].max_n;
    j->footprint = tsizes[tmpl].slot_bytes;
    if (cfg.mode == SET_MODE_SET) {
      std::unique_lock<std::mutex> lk(stage_mu);
      if ((int)staging.size() >= staging_cap && serve_ref == -1) {
        if (flags & SET_NONBLOCK) {
          lk.unlock();
          free_job(j);
          return SET_EAGAIN;
        }
        stage_room_cv.wait(lk, [&] { return (int)staging.size() < staging_cap || stopping.load(); });
        if (stopping.load()) {
          lk.unlock();
          free_job(j);
          return SET_ECLOSED;
        }
      }
      j->id = c_next.fetch_add(1);
      j->t_submit = now_ns();
      uint64_t zero = 0;
      t_first_submit.compare_exchange_strong(zero, j->t_submit);
      staging.push_back(j);
      if (id_out) *id_out = j->id;
      lk.unlock();
      stage_cv.notify_one();
      return SET_OK;
    }
    if (cfg.mode == SET_MODE_QUEUE) {
      std::lock_guard<std::mutex> g(gq_mu);
      j->id = c_next.fetch_add(1);
      j->t_submit = now_ns();
      uint64_t zero = 0;
      t_first_submit.compare_exchange_strong(zero, j->t_submit);
      if (id_out) *id_out = j->id;
      gq.push_back(j);
      return SET_OK;
    }
    std::lock_guard<std::mutex> g(base_mu);
    j->id = c_next.fetch_add(1);
    j->t_submit = now_ns();
    uint64_t zero = 0;
    t_first_submit.compare_exchange_strong(zero, j->t_submit);
    if (id_out) *id_out = j->id;
    if (cfg.mode == SET_MODE_BATCH_SYNC) {
      batch.push_back(j);
      const int bs = cfg.batch_size > 0 ? cfg.batch_size : b;
      if ((int)batch.size() >= bs) return run_batch_locked();
      return SET_OK;
    }
    // SYNC / GRAPH: run now on the next stream (round robin)
    const int si = (int)(rr_stream++ % (uint64_t)b);
    j->worker = si;
    j->slot = 0;
    j->seq = ++slot_seq[tmpl][(size_t)si * d];
    j->t_launch = now_ns();
    ++st_launch[si];
    std::string err;
    const uint64_t t0 = now_ns();
    int rc = (cfg.mode == SET_MODE_SYNC) ? be->run_sync(j, si, &err) : be->run_graph(j, si, &err);
    st_ns_launch += now_ns() - t0;
    if (rc != SET_OK) fail(rc, "run: " + err);
    record_done(j, rc);
    free_job(j);
    {
      std::lock_guard<std::mutex> g2(done_mu);
      c_done.fetch_add(1);
    }
    done_cv.notify_all();
    return rc;
  }

  int run_batch_locked() {
    if (batch.empty()) return SET_OK;
    const int n = (int)batch.size();
    for (int i = 0; i < n; ++i) {  // chain i: slot i / b of worker i % b (the backend maps it the same way)
      JobRec* j = batch[i];
      j->worker = i % b;
      j->slot = i / b;
      j->seq = ++slot_seq[j->tmpl][(size_t)j->worker * d + j->slot];
      j->t_launch = now_ns();
      ++st_launch[j->worker];
    }
    std::string err;
    const uint64_t t0 = now_ns();
    int rc = be->run_batch(batch.data(), n, &err);
    st_ns_launch += now_ns() - t0;
    ++st_batches;
    if (rc != SET_OK) fail(rc, "batch: " + err);
    for (JobRec* j : batch) {
      record_done(j, rc);
      free_job(j);
    }
    {
      std::lock_guard<std::mutex> g2(done_mu);
      c_done.fetch_add((uint64_t)n);
    }
    done_cv.notify_all();
    batch.clear();
    return rc;
  }

  // ------------------------------------------------------------------ bucketed persistent batching
  int run_vector_jobs(int tmpl, const set_vec_job* jobs, uint64_t count, float* results, const set_vec_tuning* tune,
                      uint64_t* nbatches_out) {
    int st = check_sticky();
    if (st != SET_OK) return st;
    if (!valid_template(tmpl)) return fail(SET_EINVAL, "unknown template id");
    const set_job_template& t = templates[tmpl];
    if (t.pipeline != SET_PIPE_SAXPY_BATCH_F32) return fail(SET_EINVAL, "template is not a vector batch template");
    if (count && (!jobs || !results)) return fail(SET_EINVAL, "null jobs or results");
    std::vector<std::vector<uint32_t>> buckets(64);
    for (uint64_t i = 0; i < count; ++i) {
      const set_vec_job& j = jobs[i];
      if (j.n < 1 || j.n > t.max_n) return fail(SET_EINVAL, "vector job n outside [1, max_n]");
      if (j.x_off > t.pool_len || j.n > t.pool_len - j.x_off || j.y_off > t.pool_len || j.n > t.pool_len - j.y_off)
        return fail(SET_EINVAL, "vector job window outside the pool");
      buckets[63 - __builtin_clzll(j.n)].push_back((uint32_t)i);
    }
    struct Plan {
      uint32_t te, grid;
      std::vector<uint32_t> idx;
      uint32_t tiles;
    };
    std::vector<Plan> plans;
    for (int bk = 0; bk < 64; ++bk) {
      if (buckets[bk].empty()) continue;
      uint32_t te = (tune && tune->tile_elems[bk]) ? tune->tile_elems[bk] : vec_default_tile(bk);
      uint32_t grid = (tune && tune->grid[bk]) ? tune->grid[bk] : (t.grid > 0 ? (uint32_t)t.grid : kVecBatchGrid);
      if (te % 1024 != 0 || grid < 1) return fail(SET_EINVAL, "tile_elems must be a positive multiple of 1024");
      Plan cur{te, grid, {}, 0};
      for (uint32_t i : buckets[bk]) {
        const uint64_t nt = (jobs[i].n + te - 1) / te;
        if (nt > t.tiles_max) return fail(SET_EINVAL, "a job needs more work items than tiles_max");
        if (cur.idx.size() >= t.batch_max || cur.tiles + nt > t.tiles_max) {
          plans.push_back(std::move(cur));
          cur = Plan{te, grid, {}, 0};
        }
        cur.idx.push_back(i);
        cur.tiles += (uint32_t)nt;
      }
      if (!cur.idx.empty()) plans.push_back(std::move(cur));
    }
    auto up64 = [](uint64_t v) { return (v + 63) / 64 * 64; };
    uint64_t total = 0;
    for (const Plan& pl : plans) total += up64(64 + 48ull * pl.idx.size()) + up64(64 + 4ull * pl.idx.size());
    if (plans.empty()) {
      if (nbatches_out) *nbatches_out = 0;
      return SET_OK;
    }
    // Pinned staging for the tables and results: kept by the context and
    // grown when a call needs more, so repeated calls allocate nothing.
    std::lock_guard<std::mutex> vg(vec_stage_mu);
    if (vec_stage_bytes < total) {
      if (vec_stage) be->free_host(vec_stage);
      vec_stage_bytes = 0;
      vec_stage = (char*)be->alloc_host(total);
      if (!vec_stage) return fail(SET_ENOMEM, "pinned staging for descriptor tables");
      vec_stage_bytes = total;
    }
    char* stage_mem = vec_stage;
    std::vector<char*> outs(plans.size());
    uint64_t off = 0;
    int rc = SET_OK;
    for (size_t k = 0; k < plans.size() && rc == SET_OK; ++k) {
      const Plan& pl = plans[k];
      const uint32_t c = (uint32_t)pl.idx.size();
      char* tab = stage_mem + off;
      off += up64(64 + 48ull * c);
      outs[k] = stage_mem + off;
      off += up64(64 + 4ull * c);
      VecBatchHdr* H = reinterpret_cast<VecBatchHdr*>(tab);
      std::memset(H, 0, sizeof(*H));
      H->count = c;
      H->total_tiles = pl.tiles;
      VecBatchDesc* D = reinterpret_cast<VecBatchDesc*>(tab + sizeof(VecBatchHdr));
      uint32_t ts = 0;
      for (uint32_t q = 0; q < c; ++q) {
        const set_vec_job& j = jobs[pl.idx[q]];
        D[q].x_off = j.x_off;
        D[q].y_off = j.y_off;
        D[q].n = (uint32_t)j.n;
        D[q].a = j.a;
        D[q].tile_start = ts;
        D[q].ntiles = (uint32_t)((j.n + pl.te - 1) / pl.te);
        D[q].tile_elems = pl.te;
        D[q].pad[0] = D[q].pad[1] = D[q].pad[2] = 0;
        ts += D[q].ntiles;
      }
      set_job_args a;
      std::memset(&a, 0, sizeof(a));
      a.host_in = tab;
      a.in_bytes = 64 + 48ull * c;
      a.host_out = outs[k];
      a.out_bytes = 64 + 4ull * c;
      a.n = c;
      a.worker_hint = -1;
      a.grid = pl.grid;
      a.user_tag = k;
      rc = submit(tmpl, &a, 0, nullptr);
    }
    int drc = drain(-1);
    if (rc == SET_OK) rc = drc;
    if (rc == SET_OK) {
      for (size_t k = 0; k < plans.size(); ++k) {
        const set_out_header* h = reinterpret_cast<const set_out_header*>(outs[k]);
        if (h->magic != SET_OUT_MAGIC || h->canary_ok != 1 || h->user_tag != k) {
          rc = fail(SET_EDEVICE, "vector batch output header check failed");
          break;
        }
        const float* r = reinterpret_cast<const float*>(outs[k] + 64);
        for (size_t q = 0; q < plans[k].idx.size(); ++q) results[plans[k].idx[q]] = r[q];
      }
    }
    if (nbatches_out) *nbatches_out = plans.size();
    return rc;
  }

  // Vector requests -> batches, whenever a batch slot is free (continuous batching).
  void serve_batcher() {
    ServeState& S = *serve_st;
    const set_job_template& t = templates[S.vtmpl];
    while (true) {
      int r = -1;
      std::vector<uint32_t> take;
      {
        std::unique_lock<std::mutex> lk(S.mu);
        S.cv.wait(lk, [&] {
          return (!S.pending.empty() && S.inflight < S.vec_inflight_max) || (S.arrivals_done && S.pending.empty()) ||
                 check_sticky() != SET_OK;
        });
        if (S.pending.empty() || check_sticky() != SET_OK) {
          if (S.arrivals_done || check_sticky() != SET_OK) return;
          continue;
        }
        for (size_t k = 0; k < S.ring.size(); ++k)
          if (!S.ring[k].busy) {
            r = (int)k;
            break;
          }
        uint64_t tiles = 0;
        while (!S.pending.empty() && take.size() < S.vec_batch_max) {
          const set_job_args& a = S.reqs[S.pending.front()].args;
          const int bk = 63 - __builtin_clzll(a.n);
          const uint32_t te = (S.tuning && S.tuning->tile_elems[bk]) ? S.tuning->tile_elems[bk] : vec_default_tile(bk);
          const uint64_t nt = (a.n + te - 1) / te;
          if (!take.empty() && tiles + nt > t.tiles_max) break;
          tiles += nt;
          take.push_back(S.pending.front());
          S.pending.pop_front();
        }
        S.ring[r].busy = true;
        S.ring[r].idx = take;
        ++S.inflight;
      }
      VecRing& R = S.ring[r];
      VecBatchHdr* H = reinterpret_cast<VecBatchHdr*>(R.tab);
      std::memset(H, 0, sizeof(*H));
      VecBatchDesc* D = reinterpret_cast<VecBatchDesc*>(R.tab + sizeof(VecBatchHdr));
      uint32_t ts = 0;
      for (size_t q = 0; q < take.size(); ++q) {
        const set_job_args& a = S.reqs[take[q]].args;
        const int bk = 63 - __builtin_clzll(a.n);
        const uint32_t te = (S.tuning && S.tuning->tile_elems[bk]) ? S.tuning->tile_elems[bk] : vec_default_tile(bk);
        D[q].x_off = a.x_off;
        D[q].y_off = a.y_off;
        D[q].n = (uint32_t)a.n;
        D[q].a = a.a;
        D[q].tile_start = ts;
        D[q].ntiles = (uint32_t)((a.n + te - 1) / te);
        D[q].tile_elems = te;
        D[q].pad[0] = D[q].pad[1] = D[q].pad[2] = 0;
        ts += D[q].ntiles;
      }
      H->count = (uint32_t)take.size();
      H->total_tiles = ts;
      set_job_args b;
      std::memset(&b, 0, sizeof(b));
      b.host_in = R.tab;
      b.in_bytes = 64 + 48ull * take.size();
      b.host_out = R.res;
      b.out_bytes = 64 + 4ull * take.size();
      b.n = take.size();
      b.worker_hint = -1;
      ++S.batches;
      if (submit(S.vtmpl, &b, 0, nullptr, -2 - (int64_t)r) != SET_OK) {
        std::lock_guard<std::mutex> g(S.mu);
        S.failed += take.size();
        R.busy = false;
        --S.inflight;
      }
    }
  }

  int serve(const set_request* reqs, uint64_t count, const set_serve_config* cfgp, uint64_t* done_ns,
            float* vec_results, set_serve_stats* out) {
    int st = check_sticky();
    if (st != SET_OK) return st;
    if (cfg.mode != SET_MODE_SET) return fail(SET_EUNSUPPORTED, "set_serve needs SET mode");
    if (count && (!reqs || !done_ns)) return fail(SET_EINVAL, "null requests or done_ns");
    set_serve_config sc{};
    if (cfgp) sc = *cfgp;
    std::unique_ptr<ServeState> S(new ServeState());
    S->reqs = reqs;
    S->done_ns = done_ns;
    S->vec_results = vec_results;
    S->tuning = sc.tuning;
    uint64_t nvec = 0;
    for (uint64_t i = 0; i < count; ++i) {
      const set_request& q = reqs[i];
      if (!valid_template(q.template_id)) return fail(SET_EINVAL, "unknown template id");
      if (i && q.t_arrival_ns < reqs[i - 1].t_arrival_ns) return fail(SET_EINVAL, "arrivals must be non-decreasing");
      const set_job_template& t = templates[q.template_id];
      std::string why;
      if (t.pipeline == SET_PIPE_SAXPY_BATCH_F32) {
        if (S->vtmpl >= 0 && S->vtmpl != q.template_id) return fail(SET_EINVAL, "one vector batch template per run");
        S->vtmpl = q.template_id;
        if (q.args.n < 1 || q.args.n > t.max_n || q.args.x_off > t.pool_len || q.args.n > t.pool_len - q.args.x_off ||
            q.args.y_off > t.pool_len || q.args.n > t.pool_len - q.args.y_off)
          return fail(SET_EINVAL, "vector request outside the template's limits");
        ++nvec;
      } else if (pipeline_validate_job(t, q.args, &why) != SET_OK) {
        return fail(SET_EINVAL, why);
      }
      done_ns[i] = 0;
    }
    if (nvec && !vec_results) return fail(SET_EINVAL, "vector requests need vec_results");
    char* ring_mem = nullptr;
    if (S->vtmpl >= 0) {
      const set_job_template& t = templates[S->vtmpl];
      S->vec_batch_max = sc.vec_batch_max ? std::min(sc.vec_batch_max, t.batch_max) : t.batch_max;
      S->vec_inflight_max = sc.vec_inflight ? sc.vec_inflight : (uint32_t)b;
      const uint64_t tb = (64 + 48ull * S->vec_batch_max + 255) / 256 * 256;
      const uint64_t rb = (64 + 4ull * S->vec_batch_max + 255) / 256 * 256;
      ring_mem = (char*)be->alloc_host((tb + rb) * S->vec_inflight_max);
      if (!ring_mem) return fail(SET_ENOMEM, "pinned staging for vector batches");
      S->ring.resize(S->vec_inflight_max);
      for (uint32_t k = 0; k < S->vec_inflight_max; ++k) {
        S->ring[k].tab = ring_mem + (tb + rb) * k;
        S->ring[k].res = S->ring[k].tab + tb;
      }
    }
    serve_st = S.get();
    std::thread batcher;
    if (S->vtmpl >= 0) batcher = std::thread([this] { serve_batcher(); });
    uint64_t arrived = 0, max_backlog = 0;
    int rc = SET_OK;
    S->t0 = now_ns();
    for (uint64_t i = 0; i < count; ++i) {
      const set_request& q = reqs[i];
      if (sc.window_ns && q.t_arrival_ns > sc.window_ns) break;
      const uint64_t target = S->t0 + q.t_arrival_ns;
      uint64_t now = now_ns();
      while (now < target) {
        if (target - now > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(target - now - 100000));
        now = now_ns();
      }
      ++arrived;
      uint64_t backlog = 0;
      {
        std::lock_guard<std::mutex> g(stage_mu);
        backlog = staging.size();
      }
      if (q.template_id == S->vtmpl) {
        std::lock_guard<std::mutex> g(S->mu);
        S->pending.push_back((uint32_t)i);
        backlog += S->pending.size();
      } else {
        rc = submit(q.template_id, &q.args, 0, nullptr, (int64_t)i);
        if (rc != SET_OK) break;
      }
      max_backlog = std::max(max_backlog, backlog);
      if (q.template_id == S->vtmpl) S->cv.notify_all();
    }
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->arrivals_done = true;
    }
    S->cv.notify_all();
    if (batcher.joinable()) batcher.join();
    const int drc = drain(-1);
    if (rc == SET_OK) rc = drc;
    serve_st = nullptr;
    if (ring_mem) be->free_host(ring_mem);
    if (out) {
      std::memset(out, 0, sizeof(*out));
      out->arrived = arrived;
      out->completed = S->completed.load();
      out->failed = S->failed.load();
      out->not_admitted = count - arrived;
      out->vec_batches = S->batches.load();
      out->t_start_ns = S->t0;
      out->t_end_ns = S->t0 + S->t_last.load();
      out->max_backlog = max_backlog;
    }
    return rc;
  }

  int drain(int64_t timeout_ns) {
    if (cfg.mode == SET_MODE_BATCH_SYNC) {
      std::lock_guard<std::mutex> g(base_mu);
      run_batch_locked();
    }
    std::unique_lock<std::mutex> lk(done_mu);
    auto pred = [&] { return c_done.load() >= c_next.load(); };
    if (timeout_ns < 0) {
      done_cv.wait(lk, pred);
    } else if (!timed_wait(done_cv, lk, std::chrono::nanoseconds(timeout_ns), pred)) {
      return SET_ETIMEOUT;
    }
    return check_sticky();
  }

  void stats(set_stats* o) {
    std::memset(o, 0, sizeof(*o));
    o->submitted = c_next.load() - submitted_base.load();
    o->completed = st_completed.load();
    o->stolen = st_stolen.load();
    o->failed = st_failed.load();
    for (int i = 0; i < kStatWorkers; ++i) o->launches_per_worker[i] = st_launch[i].load();
    o->host_ns_bind = st_ns_bind.load();
    o->host_ns_launch = st_ns_launch.load();
    o->host_ns_callback = st_ns_cb.load();
    o->host_ns_sync = be ? be->host_ns_sync() : 0;
    o->queue_high_water = st_q_hw.load();
    o->inflight_high_water = st_inflight_hw.load();
    o->bytes_h2d = st_h2d.load();
    o->bytes_d2h = st_d2h.load();
    o->mem_in_use = mem_in_use.load();
    o->mem_high_water = st_mem_hw.load();
    o->batches = st_batches.load();
    o->t_first_submit_ns = t_first_submit.load();
    o->t_last_done_ns = t_last_done.load();
  }

  void reset_stats() {
    submitted_base = c_next.load();
    st_completed = 0;
    st_stolen = 0;
    st_failed = 0;
    for (int i = 0; i < kMaxWorkers; ++i) st_launch[i] = 0;
    st_ns_bind = 0;
    st_ns_launch = 0;
    st_ns_cb = 0;
    st_q_hw = 0;
    st_inflight_hw = 0;
    st_h2d = 0;
    st_d2h = 0;
    st_mem_hw = mem_in_use.load();
    st_batches = 0;
    t_first_submit = 0;
    t_last_done = 0;
    std::lock_guard<std::mutex> g(times_mu);
    times.clear();
  }
};

}  // namespace setrt

using setrt::Context;

struct set_ctx {
  Context impl;
};

extern "C" {

const char* set_strerror(int code) {
  switch (code) {
    case SET_OK: return "SET_OK";
    case SET_EINVAL: return "SET_EINVAL";
    case SET_ENOMEM: return "SET_ENOMEM";
    case SET_EDEVICE: return "SET_EDEVICE";
    case SET_EAGAIN: return "SET_EAGAIN";
    case SET_ETIMEOUT: return "SET_ETIMEOUT";
    case SET_ECLOSED: return "SET_ECLOSED";
    case SET_EUNSUPPORTED: return "SET_EUNSUPPORTED";
  }
  return "SET_E?";
}

int set_ctx_create(const set_config* cfg, set_ctx** out) {
  setrt::g_create_error.clear();
  if (!cfg || !out) {
    setrt::g_create_error = "null argument";
    return SET_EINVAL;
  }
  *out = nullptr;
  if (cfg->abi_version != SET_ABI_VERSION) {
    setrt::g_create_error = "abi_version mismatch";
    return SET_EINVAL;
  }
  if (cfg->num_workers < 1 || cfg->num_workers > setrt::kMaxWorkers || cfg->slots_per_worker < 1 ||
      cfg->slots_per_worker > setrt::kMaxSlots || cfg->mode < SET_MODE_SET || cfg->mode > SET_MODE_QUEUE ||
      cfg->batch_size < 0 || cfg->batch_size > cfg->num_workers * cfg->slots_per_worker ||
      cfg->callback_mode < SET_CB_EVENT_POLL ||
      cfg->callback_mode > SET_CB_EVENT_BLOCKING || cfg->submit_policy < 0 || cfg->submit_policy > SET_SUBMIT_SKEW0 ||
      cfg->inflight_per_worker < 0 || cfg->queue_capacity < 0 || cfg->spin_us < 0 || cfg->staging_capacity < 0 ||
      cfg->dispatch_threads < 0 || cfg->dispatch_threads > setrt::kMaxThreads ||
      cfg->input_copy_streams < 0 || cfg->input_copy_streams > setrt::kMaxThreads ||
      cfg->callback_streams < 0 || cfg->callback_streams > setrt::kMaxThreads ||
      (cfg->steal_policy != SET_STEAL_ANY && cfg->steal_policy != SET_STEAL_BUSY) ||
      (cfg->backend != SET_BACKEND_HIP && cfg->backend != SET_BACKEND_FAKE)) {
    setrt::g_create_error = "invalid configuration";
    return SET_EINVAL;
  }
  set_ctx* c = new (std::nothrow) set_ctx();
  if (!c) return SET_ENOMEM;
  int rc = c->impl.init(*cfg);
  if (rc != SET_OK) {
    setrt::g_create_error = c->impl.last_error;
    delete c;
    return rc;
  }
  *out = c;
  return SET_OK;
}

int set_ctx_destroy(set_ctx* c) {
  if (!c) return SET_OK;
  if (c->impl.check_sticky() == SET_OK) c->impl.drain(-1);
  c->impl.shutdown();
  delete c;
  return SET_OK;
}

int set_template_footprint(const set_config* cfg, const set_job_template* t, uint64_t* slot_bytes,
                           uint64_t* total_bytes) {
  if (!t) return SET_EINVAL;
  setrt::TemplateSizes sz;
  if (setrt::pipeline_sizes(*t, &sz) != SET_OK) return SET_EINVAL;
  if (slot_bytes) *slot_bytes = sz.slot_bytes;
  if (total_bytes) {
    if (!cfg) return SET_EINVAL;
    *total_bytes = sz.slot_bytes * (uint64_t)cfg->num_workers * (uint64_t)cfg->slots_per_worker;
  }
  return SET_OK;
}

int set_template_define(set_ctx* c, const set_job_template* t, int* template_id) {
  if (!c || !t || !template_id) return SET_EINVAL;
  int st = c->impl.check_sticky();
  if (st != SET_OK) return st;
  return c->impl.define_template(*t, template_id);
}

int set_submit(set_ctx* c, int template_id, const set_job_args* a, int flags, uint64_t* job_id) {
  if (!c) return SET_EINVAL;
  return c->impl.submit(template_id, a, flags, job_id);
}

int set_submit_many(set_ctx* c, int template_id, const set_job_args* a, uint64_t count, int flags,
                    uint64_t* first_job_id) {
  if (!c || (!a && count)) return SET_EINVAL;
  for (uint64_t i = 0; i < count; ++i) {
    uint64_t id = 0;
    int rc = c->impl.submit(template_id, a + i, flags, &id);
    if (rc != SET_OK) return rc;
    if (i == 0 && first_job_id) *first_job_id = id;
  }
  return SET_OK;
}

int set_set_completion_cb(set_ctx* c, set_completion_fn fn, void* user) {
  if (!c) return SET_EINVAL;
  c->impl.user_arg.store(user);
  c->impl.user_fn.store(fn);
  return SET_OK;
}

int set_drain(set_ctx* c, int64_t timeout_ns) {
  if (!c) return SET_EINVAL;
  return c->impl.drain(timeout_ns);
}

int set_get_stats(set_ctx* c, set_stats* out) {
  if (!c || !out) return SET_EINVAL;
  c->impl.stats(out);
  return SET_OK;
}

int set_reset_stats(set_ctx* c) {
  if (!c) return SET_EINVAL;
  c->impl.reset_stats();
  return SET_OK;
}

int set_get_job_times(set_ctx* c, set_job_times* out, uint64_t max, uint64_t* count) {
  if (!c || !count || (!out && max)) return SET_EINVAL;
  std::lock_guard<std::mutex> g(c->impl.times_mu);
  const uint64_t n = std::min<uint64_t>(max, c->impl.times.size());
  if (n) std::memcpy(out, c->impl.times.data(), n * sizeof(set_job_times));
  *count = n;
  return SET_OK;
}

int set_time_stage(set_ctx* c, int template_id, int stage, int worker, int reps, double* avg_us) {
  if (!c || !avg_us || reps < 1) return SET_EINVAL;
  int st = c->impl.check_sticky();
  if (st != SET_OK) return st;
  if (!c->impl.valid_template(template_id)) return SET_EINVAL;
  if (stage != SET_STAGE_INPUT_COPY && stage != SET_STAGE_OUTPUT_COPY &&
      (stage < 0 || stage >= c->impl.tsizes[template_id].num_stages))
    return SET_EINVAL;
  if (worker < -1 || worker >= c->impl.b) return SET_EINVAL;
  std::string err;
  int rc = c->impl.be->time_stage(template_id, stage, worker, reps, avg_us, &err);
  if (rc != SET_OK) return c->impl.fail(rc, "time_stage: " + err);
  return SET_OK;
}

int set_time_device_copy(set_ctx* c, uint64_t bytes, int reps, double* avg_us) {
  if (!c || !avg_us || reps < 1 || bytes < 32 || bytes > (1ull << 30)) return SET_EINVAL;
  int st = c->impl.check_sticky();
  if (st != SET_OK) return st;
  std::string err;
  int rc = c->impl.be->time_device_copy(bytes, reps, avg_us, &err);
  if (rc != SET_OK) return c->impl.fail(rc, "time_device_copy: " + err);
  return SET_OK;
}

int set_job_io_bytes(set_ctx* c, int template_id, uint64_t n, uint64_t* in_bytes, uint64_t* out_bytes) {
  if (!c) return SET_EINVAL;
  if (!c->impl.valid_template(template_id)) return SET_EINVAL;
  const set_job_template& t = c->impl.templates[template_id];
  if (in_bytes) *in_bytes = setrt::pipeline_in_bytes(t, n);
  if (out_bytes) *out_bytes = setrt::pipeline_out_bytes(t, n);
  return SET_OK;
}

int set_stage_info(set_ctx* c, int template_id, int* num_stages, uint64_t* bytes_per_stage, int max_stages,
                   char* names, int names_len) {
  if (!c || !num_stages) return SET_EINVAL;
  if (!c->impl.valid_template(template_id)) return SET_EINVAL;
  const setrt::TemplateSizes& sz = c->impl.tsizes[template_id];
  *num_stages = sz.num_stages;
  for (int i = 0; i < sz.num_stages && i < max_stages; ++i)
    if (bytes_per_stage) bytes_per_stage[i] = sz.stage_bytes[i];
  if (names && names_len > 0) {
    std::string s;
    for (int i = 0; i < sz.num_stages; ++i) {
      if (i) s += ",";
      s += sz.stage_names[i];
    }
    snprintf(names, (size_t)names_len, "%s", s.c_str());
  }
  return SET_OK;
}

int set_run_vector_jobs(set_ctx* c, int template_id, const set_vec_job* jobs, uint64_t count, float* results,
                        const set_vec_tuning* tuning, uint64_t* batches) {
  if (!c) return SET_EINVAL;
  return c->impl.run_vector_jobs(template_id, jobs, count, results, tuning, batches);
}

int set_serve(set_ctx* c, const set_request* reqs, uint64_t count, const set_serve_config* cfg, uint64_t* done_ns,
              float* vec_results, set_serve_stats* stats) {
  if (!c) return SET_EINVAL;
  return c->impl.serve(reqs, count, cfg, done_ns, vec_results, stats);
}

const char* set_last_error(const set_ctx* c) {
  if (!c) return setrt::g_create_error.c_str();
  return c->impl.last_error.c_str();
}

}  // extern "C"
