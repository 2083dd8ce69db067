// HIP backend: job templates become per-(worker, slot) graph executables
// (H2D memcpy node -> stage kernel nodes -> D2H memcpy node, Section 4.1),
// bound per job by updating the executable's memcpy endpoints and the first
// kernel's argument block (UpdateGraphParams), launched on the worker's
// stream with a completion callback (GraphLaunch + AddCallback, Algorithm 2).
// The same slots and kernels serve the comparison systems of Section 5.1
// (direct launches, per-job graph relaunch, one batch graph of b chains).
#include <hip/hip_runtime.h>

#include <cstring>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>
#include <vector>

#include "kernels.hpp"

namespace setrt {

namespace {

#define HIPCK(expr)                                                                  \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      if (err) *err = std::string(#expr) + " failed: " + hipGetErrorString(e_);     \
      return SET_EDEVICE;                                                            \
    }                                                                                \
  } while (0)

struct CbCtx {
  JobRec* job;
  DoneFn done;
  void* ctx;
};

struct ChainNodes {
  hipGraphNode_t h2d = nullptr, d2h = nullptr, flag = nullptr;
  hipGraphNode_t delay = nullptr, poison = nullptr;  // memory-safety stress nodes (template options)
  hipGraphNode_t k[kMaxStages] = {};
};

struct Slot {
  char* base = nullptr;
  int tmpl = 0, w = 0, s = 0;
  BoxArgs box;
  Div9Args div;
  HistArgs hist;
  HistFinalArgs histf;
  GaussArgs gauss;
  SobelArgs sobel;
  SobelFinalArgs sobelf;
  VecArgs vec;
  VecFinalArgs vecf;
  ScanReduceArgs scan_r;
  ScanSpineArgs scan_s;
  ScanDownArgs scan_d;
  VecBatchArgs vb;
  VecBatchFinalArgs vbf;
  CopyArgs h2d_copy, d2h_copy;
  void* h2d_argv[1] = {&h2d_copy};
  void* d2h_argv[1] = {&d2h_copy};
  DoneFlagArgs flag{};
  void* flag_argv[1] = {&flag};
  PoisonArgs poison{};
  void* poison_argv[1] = {&poison};
  DelayArgs delay{};
  void* delay_argv[1] = {&delay};
  JobBeginArgs jb{};
  JobEndArgs je{};
  HotspotArgs hot[kMaxHotspotSteps] = {};
  void* lib_ws = nullptr;  // library-call templates: this slot's share of the library workspace
  size_t lib_ws_bytes = 0;
  uint64_t flag_seq = 0;  // sequence number the completion word will hold when the launched job is done
  int nstages = 0;
  const void* func[kMaxStages] = {};
  dim3 grid[kMaxStages];
  unsigned block[kMaxStages] = {};  // threads per block of each stage
  void* argv[kMaxStages][1] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ChainNodes nodes;
  hipEvent_t ev = nullptr;
  hipEvent_t in_ev = nullptr;  // end of the input copy on an input-copy stream
  bool in_prefetched = false;  // SET mode: the bound job's input copy was issued at bind
  bool in_stale = false;       // a prefetched copy of a job stolen from this slot may still be landing
  CbCtx cb{};
  const void* host_in = nullptr;
  uint64_t in_bytes = 0;
  void* host_out = nullptr;
  uint64_t out_bytes = 0;
};

struct BatchGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  std::vector<ChainNodes> chains;
};

struct Pipe {
  set_job_template t{};
  SlotLayout L{};
  char* arena = nullptr;
  bool own_arena = false;
  void* placeholder = nullptr;  // pinned host buffer the memcpy nodes point at before the first bind
  uint64_t* words = nullptr;    // completion words, one 64-byte line per slot (SET_CB_HOST_FLAG)
  void* lib_ws = nullptr;       // library-call templates: temporary storage of every slot
  std::vector<Slot> slots;      // [w * d + s]
  std::vector<BatchGraph> batch;  // [count - 1]
};

// Taps of the sampled Gaussian of radius 2 and sigma 1, normalised and
// rounded to float32: out[0] for |k| = 2, out[1] for |k| = 1, out[2] centre.
void gaussian_taps(float out[3]) {
  const double e2 = std::exp(-2.0), e1 = std::exp(-0.5), e0 = 1.0;
  const double s = e0 + 2.0 * e1 + 2.0 * e2;
  out[0] = (float)(e2 / s);
  out[1] = (float)(e1 / s);
  out[2] = (float)(e0 / s);
}

inline dim3 to_dim3(Grid3 g) { return dim3(g.x, g.y, g.z); }

// Copy mechanisms of a template: the input by copy kernel, by a graph memcpy
// node, or by hipMemcpyAsync ahead of the graph; the output by copy kernel or
// graph memcpy node.
inline bool in_by_kernel(const set_job_template& t) { return t.copy_mode == SET_COPY_KERNELS; }
inline bool in_ahead(const set_job_template& t) { return t.copy_mode == SET_COPY_ASYNC_IN; }
inline bool out_by_kernel(const set_job_template& t) { return t.copy_mode != SET_COPY_NODES; }

// Templates whose middle stage is a library call captured into the job
// graph (between stage kernel 0 and stage kernel 1).
inline bool lib_template(const set_job_template& t) { return t.pipeline == SET_PIPE_SCAN_LIB_I32_I64; }


thread_local int t_dev = -1;

class HipBackend : public Backend {
 public:
  ~HipBackend() override { shutdown(); }

  int init(const set_config& cfg, std::string* err) override {
    cfg_ = cfg;
    b_ = cfg.num_workers;
    d_ = cfg.slots_per_worker;
    int ndev = 0;
    HIPCK(hipGetDeviceCount(&ndev));
    if (cfg.device < 0 || cfg.device >= ndev) {
      if (err) *err = "no such HIP device";
      return SET_EDEVICE;
    }
    dev_ = cfg.device;
    int khz = 0;
    HIPCK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev_));
    clock_khz_ = khz > 0 ? (uint64_t)khz : 100000;
    pipes_.reserve(kMaxTemplates);  // entries never move while jobs of other templates run
    HIPCK(hipSetDevice(dev_));
    t_dev = dev_;
    streams_.resize(b_);
    if (cfg.streams) {
      for (int i = 0; i < b_; ++i) {
        if (!cfg.streams[i]) {
          if (err) *err = "null borrowed stream";
          return SET_EINVAL;
        }
        streams_[i] = (hipStream_t)cfg.streams[i];
      }
    } else {
      own_streams_ = true;
      for (int i = 0; i < b_; ++i) HIPCK(hipStreamCreateWithFlags(&streams_[i], hipStreamNonBlocking));
    }
    // Templates are defined (captured, instantiated, uploaded) on a stream of
    // their own: a capture on a worker stream would also record the job
    // launches other threads issue onto it meanwhile.
    HIPCK(hipStreamCreateWithFlags(&define_stream_, hipStreamNonBlocking));
    copy_streams_.resize(std::min(cfg.input_copy_streams, b_));
    for (hipStream_t& cs : copy_streams_) HIPCK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    if (cfg.mode == SET_MODE_SET && cfg.callback_mode == SET_CB_EVENT_CHAIN) {
      cb_streams_.resize((size_t)std::min(b_, std::max(1, cfg.callback_streams)));
      for (hipStream_t& cs : cb_streams_) HIPCK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      cb_mu_.reset(new std::mutex[cb_streams_.size()]);
    }
    flag_mode_ = cfg.mode == SET_MODE_SET && cfg.callback_mode == SET_CB_HOST_FLAG;
    if (cfg.mode == SET_MODE_SET && (cfg.callback_mode == SET_CB_EVENT_POLL || flag_mode_)) {
      poll_in_.resize(b_);
      poller_ = std::thread([this] { poll_loop(); });
    }
    blocking_ = cfg.mode == SET_MODE_SET && cfg.callback_mode == SET_CB_EVENT_BLOCKING;
    if (blocking_) {
      waiters_.resize(b_);
      for (int w = 0; w < b_; ++w) {
        waiters_[w].reset(new Waiter());
        waiters_[w]->th = std::thread([this, w] { wait_loop(w); });
      }
    }
    return SET_OK;
  }

  int define_template(int id, const set_job_template& t, std::string* err) override {
    ensure_dev();
    if ((int)pipes_.size() != id) {
      if (err) *err = "template ids out of order";
      return SET_EINVAL;
    }
    pipes_.emplace_back(new Pipe());
    Pipe& p = *pipes_.back();
    p.t = t;
    p.L = slot_layout(t);
    const uint64_t total = p.L.total * (uint64_t)b_ * (uint64_t)d_;
    if (t.arena) {
      if (t.arena_bytes < total) {
        if (err) *err = "borrowed arena smaller than the template footprint";
        return SET_ENOMEM;
      }
      p.arena = (char*)t.arena;
    } else {
      void* a = nullptr;
      hipError_t e = hipMalloc(&a, total);
      if (e != hipSuccess) {
        if (err) *err = std::string("hipMalloc arena: ") + hipGetErrorString(e);
        return SET_ENOMEM;
      }
      p.arena = (char*)a;
      p.own_arena = true;
    }
    HIPCK(hipMemset(p.arena, 0, total));
    const uint64_t ph = std::max<uint64_t>(std::max(p.L.in_cap, p.L.out_cap), 64);
    HIPCK(hipHostMalloc(&p.placeholder, ph, hipHostMallocDefault));
    std::memset(p.placeholder, 0, ph);
    if (flag_mode_) {
      HIPCK(hipHostMalloc((void**)&p.words, (size_t)b_ * d_ * 64, hipHostMallocDefault));
      std::memset(p.words, 0, (size_t)b_ * d_ * 64);
    }
    float taps[3];
    gaussian_taps(taps);
    size_t lib_ws_bytes = 0;
    if (lib_template(t)) {
      HIPCK(lib_scan(nullptr, lib_ws_bytes, nullptr, nullptr, (size_t)t.max_n, nullptr));
      lib_ws_bytes = (std::max<size_t>(lib_ws_bytes, 256) + 255) / 256 * 256;
      HIPCK(hipMalloc(&p.lib_ws, lib_ws_bytes * (size_t)b_ * d_));
    }
    p.slots.resize((size_t)b_ * d_);
    if (poisons(p)) HIPCK(hipDeviceSynchronize());  // the zero fill above, before the poison fill
    for (int w = 0; w < b_; ++w) {
      for (int s = 0; s < d_; ++s) {
        Slot& sl = p.slots[(size_t)w * d_ + s];
        sl.tmpl = id;
        sl.w = w;
        sl.s = s;
        sl.base = p.arena + p.L.total * ((uint64_t)w * d_ + s);
        setup_slot(p, sl, taps);
        if (poisons(p)) HIPCK(launch_stress(p, sl, true, define_stream_));  // a slot's first job finds poison too
        if (p.lib_ws) {
          sl.lib_ws = (char*)p.lib_ws + lib_ws_bytes * ((size_t)w * d_ + s);
          sl.lib_ws_bytes = lib_ws_bytes;
        }
        if (p.words) sl.flag = DoneFlagArgs{reinterpret_cast<const DevSlotHdr*>(sl.base + p.L.hdr),
                                            p.words + ((size_t)w * d_ + s) * 8};
        if (!copy_streams_.empty() && in_ahead(t) && (cfg_.mode == SET_MODE_SET || s == 0))
          HIPCK(hipEventCreateWithFlags(&sl.in_ev, hipEventDisableTiming));
        const uint64_t ch = canary_value(id, w, s, 0), ct = canary_value(id, w, s, 1);
        HIPCK(hipMemcpy(sl.base + p.L.hdr, &ch, 8, hipMemcpyHostToDevice));
        HIPCK(hipMemcpy(sl.base + p.L.tail, &ct, 8, hipMemcpyHostToDevice));
      }
    }
    if (cfg_.mode == SET_MODE_SET || cfg_.mode == SET_MODE_GRAPH || cfg_.mode == SET_MODE_QUEUE) {
      const int ds = (cfg_.mode == SET_MODE_SET) ? d_ : 1;
      for (int w = 0; w < b_; ++w) {
        for (int s = 0; s < ds; ++s) {
          Slot& sl = p.slots[(size_t)w * d_ + s];
          int rc;
          if ((t.flags & SET_TF_CAPTURE) || lib_template(t)) {
            rc = capture_chain(p, sl, define_stream_, &sl.graph, &sl.nodes, err);
          } else {
            HIPCK(hipGraphCreate(&sl.graph, 0));
            rc = add_chain(p, sl, sl.graph, &sl.nodes, err);
          }
          if (rc != SET_OK) return rc;
          HIPCK(hipGraphInstantiateWithFlags(&sl.exec, sl.graph, 0));
          HIPCK(hipGraphUpload(sl.exec, define_stream_));
          if (cfg_.mode == SET_MODE_SET || cfg_.mode == SET_MODE_QUEUE)
            HIPCK(hipEventCreateWithFlags(&sl.ev, blocking_ ? (hipEventDisableTiming | hipEventBlockingSync)
                                                            : hipEventDisableTiming));
        }
      }
    }
    if (cfg_.mode == SET_MODE_BATCH_SYNC) p.batch.resize((size_t)b_ * d_);
    HIPCK(hipStreamSynchronize(define_stream_));
    return SET_OK;
  }

  int bind(JobRec* j, std::string* err) override {
    ensure_dev();
    Pipe& p = *pipes_[j->tmpl];
    Slot& sl = p.slots[(size_t)j->worker * d_ + j->slot];
    set_scalars(p, sl, j);
    const int rc = update_exec(p, sl, sl.exec, sl.nodes, err);
    if (rc != SET_OK) return rc;
    // SET mode with input-copy streams: the input copy starts here, when the
    // job takes its FREE slot (nothing reads that slot's input any more), so
    // it overlaps the jobs ahead of it on the worker and is usually complete
    // when the graph is launched.  A stolen job's copy is left to its launch,
    // on the thief's own stream, rather than queued behind the copy stream's
    // backlog.
    // A slot still marked prefetched was left by a job stolen before launch,
    // whose copy may not have landed yet.  A prefetched successor copies on
    // the same copy stream, after it; any other successor waits for that
    // copy's event before its own copy (in_stale).
    const bool stale = sl.in_prefetched;
    sl.in_prefetched = false;
    sl.in_stale = false;
    if (cfg_.mode == SET_MODE_SET && in_ahead(p.t) && sl.in_ev && sl.in_bytes && !j->stolen) {
      hipStream_t cs = copy_streams_[(size_t)j->worker % copy_streams_.size()];
      HIPCK(hipMemcpyAsync(sl.base + p.L.in, sl.host_in, sl.in_bytes, hipMemcpyHostToDevice, cs));
      HIPCK(hipEventRecord(sl.in_ev, cs));
      sl.in_prefetched = true;
    } else {
      sl.in_stale = stale;
    }
    return SET_OK;
  }

  int launch(JobRec* j, DoneFn done, void* ctx, std::string* err) override {
    ensure_dev();
    Pipe& p = *pipes_[j->tmpl];
    Slot& sl = p.slots[(size_t)j->worker * d_ + j->slot];
    const int w = j->worker;
    hipStream_t st = streams_[w];
    sl.cb = CbCtx{j, done, ctx};
    sl.flag_seq = j->seq;
    HIPCK(input_ahead(p, sl, st, w));
    HIPCK(hipGraphLaunch(sl.exec, st));
    switch (cfg_.callback_mode) {
      case SET_CB_EVENT_CHAIN: {
        HIPCK(hipEventRecord(sl.ev, st));
        // the wait and its host function stay adjacent on a callback stream
        // that several dispatcher threads share
        const size_t k = (size_t)w % cb_streams_.size();
        std::lock_guard<std::mutex> g(cb_mu_[k]);
        HIPCK(hipStreamWaitEvent(cb_streams_[k], sl.ev, 0));
        HIPCK(hipLaunchHostFunc(cb_streams_[k], &HipBackend::host_cb, &sl.cb));
        break;
      }
      case SET_CB_SAME_STREAM:
        HIPCK(hipLaunchHostFunc(st, &HipBackend::host_cb, &sl.cb));
        break;
      case SET_CB_EVENT_BLOCKING: {
        HIPCK(hipEventRecord(sl.ev, st));
        Waiter& wt = *waiters_[w];
        {
          std::lock_guard<std::mutex> g(wt.mu);
          wt.q.push_back(&sl);
        }
        wt.cv.notify_one();
        break;
      }
      case SET_CB_EVENT_POLL:
      case SET_CB_HOST_FLAG: {
        if (!flag_mode_) HIPCK(hipEventRecord(sl.ev, st));
        bool wake;
        {
          std::lock_guard<std::mutex> g(poll_mu_);
          poll_in_[w].push_back(&sl);
          poll_new_.store(true, std::memory_order_release);
          wake = poll_idle_;
        }
        if (wake) poll_cv_.notify_one();
        break;
      }
    }
    return SET_OK;
  }

  int launch_polled(JobRec* j, std::string* err) override {
    ensure_dev();
    Pipe& p = *pipes_[j->tmpl];
    Slot& sl = p.slots[(size_t)j->worker * d_ + j->slot];
    hipStream_t st = streams_[j->worker];
    HIPCK(input_ahead(p, sl, st, j->worker));
    HIPCK(hipGraphLaunch(sl.exec, st));
    HIPCK(hipEventRecord(sl.ev, st));
    return SET_OK;
  }

  int is_done(JobRec* j, bool* done, std::string* err) override {
    Pipe& p = *pipes_[j->tmpl];
    Slot& sl = p.slots[(size_t)j->worker * d_ + j->slot];
    const hipError_t e = hipEventQuery(sl.ev);
    if (e == hipSuccess) {
      *done = true;
      return SET_OK;
    }
    if (e == hipErrorNotReady) {
      *done = false;
      return SET_OK;
    }
    if (err) *err = std::string("hipEventQuery failed: ") + hipGetErrorString(e);
    return SET_EDEVICE;
  }

  int run_sync(JobRec* j, int si, std::string* err) override {
    ensure_dev();
    Pipe& p = *pipes_[j->tmpl];
    Slot& sl = p.slots[(size_t)si * d_];
    set_scalars(p, sl, j);
    hipStream_t st = streams_[si];
    if (sl.in_bytes) {
      if (in_by_kernel(p.t)) {
        sl.h2d_copy = CopyArgs{sl.host_in, sl.base + p.L.in, sl.in_bytes};
        HIPCK(hipLaunchKernel((const void*)&k_copy_in, dim3(kCopyBlocks), dim3(kBlock), sl.h2d_argv, 0, st));
      } else if (in_ahead(p.t)) {
        HIPCK(input_ahead(p, sl, st, si));
      } else {
        HIPCK(hipMemcpyAsync(sl.base + p.L.in, sl.host_in, sl.in_bytes, hipMemcpyHostToDevice, st));
      }
    }
    if (delays(p)) HIPCK(launch_stress(p, sl, false, st));
    for (int i = 0; i < sl.nstages; ++i) {
      if (i == 1) HIPCK(library_stage(p, sl, st));
      HIPCK(hipLaunchKernel(sl.func[i], sl.grid[i], dim3(sl.block[i]), sl.argv[i], 0, st));
    }
    if (out_by_kernel(p.t)) {
      sl.d2h_copy = CopyArgs{sl.base + p.L.out, sl.host_out, sl.out_bytes};
      HIPCK(hipLaunchKernel((const void*)&k_copy_out, dim3(d2h_copy_blocks(p.L.out_cap)), dim3(kBlock), sl.d2h_argv, 0, st));
    } else {
      HIPCK(hipMemcpyAsync(sl.host_out, sl.base + p.L.out, sl.out_bytes, hipMemcpyDeviceToHost, st));
    }
    if (poisons(p)) HIPCK(launch_stress(p, sl, true, st));
    const uint64_t t0 = now_ns();
    HIPCK(hipStreamSynchronize(st));
    sync_ns_ += now_ns() - t0;
    return SET_OK;
  }

  int run_graph(JobRec* j, int si, std::string* err) override {
    ensure_dev();
    Pipe& p = *pipes_[j->tmpl];
    Slot& sl = p.slots[(size_t)si * d_];
    set_scalars(p, sl, j);
    int rc = update_exec(p, sl, sl.exec, sl.nodes, err);
    if (rc != SET_OK) return rc;
    hipStream_t st = streams_[si];
    HIPCK(input_ahead(p, sl, st, si));
    HIPCK(hipGraphLaunch(sl.exec, st));
    const uint64_t t0 = now_ns();
    HIPCK(hipStreamSynchronize(st));
    sync_ns_ += now_ns() - t0;
    return SET_OK;
  }

  // Chain i of a batch graph runs in slot i / b of worker i % b (the
  // scheduler assigns the jobs' worker and slot the same way).
  Slot& batch_slot(Pipe& p, int i) { return p.slots[(size_t)(i % b_) * d_ + (size_t)(i / b_)]; }

  int run_batch(JobRec** jobs, int count, std::string* err) override {
    ensure_dev();
    if (count < 1) return SET_OK;
    const int tmpl = jobs[0]->tmpl;
    for (int i = 1; i < count; ++i)
      if (jobs[i]->tmpl != tmpl) {
        if (err) *err = "a batch graph holds chains of one template";
        return SET_EINVAL;
      }
    Pipe& p = *pipes_[tmpl];
    BatchGraph& bg = p.batch[count - 1];
    if (!bg.ex) {
      HIPCK(hipGraphCreate(&bg.g, 0));
      bg.chains.resize(count);
      for (int i = 0; i < count; ++i) {
        int rc = add_chain(p, batch_slot(p, i), bg.g, &bg.chains[i], err);
        if (rc != SET_OK) return rc;
      }
      HIPCK(hipGraphInstantiateWithFlags(&bg.ex, bg.g, 0));
      HIPCK(hipGraphUpload(bg.ex, streams_[0]));
    }
    for (int i = 0; i < count; ++i) {
      Slot& sl = batch_slot(p, i);
      set_scalars(p, sl, jobs[i]);
      int rc = update_exec(p, sl, bg.ex, bg.chains[i], err);
      if (rc != SET_OK) return rc;
      HIPCK(input_ahead(p, sl, streams_[0], i % b_));
    }
    HIPCK(hipGraphLaunch(bg.ex, streams_[0]));
    const uint64_t t0 = now_ns();
    HIPCK(hipStreamSynchronize(streams_[0]));
    sync_ns_ += now_ns() - t0;
    return SET_OK;
  }

  int time_device_copy(uint64_t bytes, int reps, double* avg_us, std::string* err) override {
    ensure_dev();
    const uint64_t half = (bytes / 2 + 15) / 16 * 16, nvec = half / 16;
    const uint64_t k = std::max<uint64_t>(2, (512ull << 20) / half);  // slices per buffer
    // a stream of its own: a template capture on the definition stream must
    // not record these launches
    hipStream_t st = nullptr;
    HIPCK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    void* buf = nullptr;
    const hipError_t ea = hipMalloc(&buf, 2 * k * half);
    if (ea != hipSuccess) {
      (void)hipStreamDestroy(st);
      if (err) *err = std::string("hipMalloc: ") + hipGetErrorString(ea);
      return SET_ENOMEM;
    }
    char* a = static_cast<char*>(buf);
    char* b = a + k * half;
    const unsigned grid = (unsigned)((nvec + kBlock - 1) / kBlock);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto once = [&](uint64_t r) {
      const uint64_t i = (r * 7 + 3) % k;  // stride through the slices so neighbours are not reused
      RefCopyArgs ra{a + i * half, b + i * half, nvec};
      void* argv[1] = {&ra};
      return hipLaunchKernel((const void*)&k_ref_copy, dim3(grid), dim3(kBlock), argv, 0, st);
    };
    hipError_t e = hipSuccess;  // the contents do not matter to a copy's timing
    for (uint64_t r = 0; e == hipSuccess && r < std::min<uint64_t>(k, 16); ++r) e = once(r + 1000);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; e == hipSuccess && r < reps; ++r) e = once((uint64_t)r);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    (void)hipStreamDestroy(st);
    if (e != hipSuccess) {
      if (err) *err = std::string("device copy: ") + hipGetErrorString(e);
      return SET_EDEVICE;
    }
    *avg_us = (double)ms * 1000.0 / reps;
    return SET_OK;
  }

  int time_stage(int tmpl, int stage, int worker, int reps, double* avg_us, std::string* err) override {
    ensure_dev();
    Pipe& p = *pipes_[tmpl];
    // worker < 0: launches rotate over every slot of the template (slot r mod
    // b*d for launch r, on worker 0's stream), so a working set larger than
    // the caches is read from HBM; otherwise slot 0 of `worker`, every launch.
    const bool rotate = worker < 0;
    const size_t nslots = rotate ? p.slots.size() : 1;
    const size_t first = rotate ? 0 : (size_t)worker * d_;
    Slot& sl0 = p.slots[first];
    // library-call templates list [stage 0, library call, stage 1]
    const bool lib = lib_template(p.t);
    const int nlisted = sl0.nstages + (lib ? 1 : 0);
    const bool copy_in = stage == SET_STAGE_INPUT_COPY, copy_out = stage == SET_STAGE_OUTPUT_COPY;
    if (!copy_in && !copy_out && (stage < 0 || stage >= nlisted)) {
      if (err) *err = "no such stage";
      return SET_EINVAL;
    }
    const bool lib_call = lib && stage == 1;
    const int ks = (lib && stage == 2) ? 1 : stage;
    hipStream_t st = streams_[rotate ? 0 : worker];
    // The copies as a job performs them (copy kernel, or DMA for memcpy nodes
    // and async input copies), of the template's largest input / output,
    // between the slot and the template's own pinned placeholder buffer.
    const uint64_t in_b = pipeline_in_bytes(p.t, 0), out_b = pipeline_out_bytes(p.t, 0);
    auto once = [&](int r) -> hipError_t {
      Slot& sl = p.slots[first + (size_t)r % nslots];
      if (copy_in) {
        if (in_b == 0) return hipSuccess;
        if (in_by_kernel(p.t)) {
          CopyArgs ca{p.placeholder, sl.base + p.L.in, in_b};
          void* av[1] = {&ca};
          return hipLaunchKernel((const void*)&k_copy_in, dim3(kCopyBlocks), dim3(kBlock), av, 0, st);
        }
        return hipMemcpyAsync(sl.base + p.L.in, p.placeholder, in_b, hipMemcpyHostToDevice, st);
      }
      if (copy_out) {
        if (out_by_kernel(p.t)) {
          CopyArgs ca{sl.base + p.L.out, p.placeholder, out_b};
          void* av[1] = {&ca};
          return hipLaunchKernel((const void*)&k_copy_out, dim3(d2h_copy_blocks(p.L.out_cap)), dim3(kBlock), av, 0, st);
        }
        return hipMemcpyAsync(p.placeholder, sl.base + p.L.out, out_b, hipMemcpyDeviceToHost, st);
      }
      if (lib_call) return library_stage(p, sl, st);
      return hipLaunchKernel(sl.func[ks], sl.grid[ks], dim3(sl.block[ks]), sl.argv[ks], 0, st);
    };
    hipEvent_t e0, e1;
    HIPCK(hipEventCreate(&e0));
    HIPCK(hipEventCreate(&e1));
    // Untimed launches first, so the timed ones start behind a queue of work
    // and the host's enqueue rate cannot pace them (a queue of twice the
    // timed launches covers a host that enqueues at up to a third of the
    // kernel's rate): the last slots before the rotation's first, or slot 0.
    const size_t ahead = std::min<size_t>(rotate ? nslots : SIZE_MAX, std::max<size_t>(64, 2 * (size_t)reps));
    for (size_t r = 0; r < ahead; ++r) HIPCK(once((int)(nslots - 1 - r % nslots)));
    HIPCK(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) HIPCK(once(r));
    HIPCK(hipEventRecord(e1, st));
    HIPCK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, e0, e1));
    HIPCK(hipEventDestroy(e0));
    HIPCK(hipEventDestroy(e1));
    *avg_us = (double)ms * 1e3 / reps;
    return SET_OK;
  }

  uint64_t host_ns_sync() const override { return sync_ns_.load(); }

  void* alloc_host(uint64_t bytes) override {
    ensure_dev();
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
  }
  void free_host(void* p) override {
    if (p) (void)hipHostFree(p);
  }

  void shutdown() override {
    if (down_) return;
    down_ = true;
    for (auto& wt : waiters_) {
      {
        std::lock_guard<std::mutex> g(wt->mu);
        wt->stop = true;
      }
      wt->cv.notify_all();
      wt->th.join();
    }
    waiters_.clear();
    if (poller_.joinable()) {
      {
        std::lock_guard<std::mutex> g(poll_mu_);
        poll_stop_ = true;
      }
      poll_cv_.notify_all();
      poller_.join();
    }
    if (dev_ >= 0) (void)hipSetDevice(dev_);
    (void)hipDeviceSynchronize();
    for (auto& pp : pipes_) {
      Pipe& p = *pp;
      for (Slot& sl : p.slots) {
        if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
        if (sl.graph) (void)hipGraphDestroy(sl.graph);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.in_ev) (void)hipEventDestroy(sl.in_ev);
      }
      for (BatchGraph& bg : p.batch) {
        if (bg.ex) (void)hipGraphExecDestroy(bg.ex);
        if (bg.g) (void)hipGraphDestroy(bg.g);
      }
      if (p.own_arena && p.arena) (void)hipFree(p.arena);
      if (p.placeholder) (void)hipHostFree(p.placeholder);
      if (p.words) (void)hipHostFree(p.words);
      if (p.lib_ws) (void)hipFree(p.lib_ws);
    }
    pipes_.clear();
    for (hipStream_t s : cb_streams_) (void)hipStreamDestroy(s);
    cb_streams_.clear();
    for (hipStream_t s : copy_streams_) (void)hipStreamDestroy(s);
    copy_streams_.clear();
    if (define_stream_) (void)hipStreamDestroy(define_stream_);
    define_stream_ = nullptr;
    if (own_streams_)
      for (hipStream_t s : streams_) (void)hipStreamDestroy(s);
    streams_.clear();
  }

 private:
  void ensure_dev() {
    if (t_dev != dev_) {
      (void)hipSetDevice(dev_);
      t_dev = dev_;
    }
  }

  static void host_cb(void* p) {
    const CbCtx c = *static_cast<CbCtx*>(p);  // copy: the slot may be rebound once done() returns
    c.done(c.ctx, c.job, SET_OK);
  }

  // Completion thread of SET_CB_EVENT_POLL and SET_CB_HOST_FLAG.  A worker's
  // jobs complete in launch order (one stream), so only the oldest pending
  // job of each worker is checked.  New launches are taken over from the
  // shared lists under the mutex; the checks themselves run without it, so
  // the dispatcher never waits on a sweep.
  bool job_done(Slot* sl) {
    if (flag_mode_) return __atomic_load_n(sl->flag.word, __ATOMIC_ACQUIRE) == sl->flag_seq;
    return hipEventQuery(sl->ev) == hipSuccess;
  }

  void poll_loop() {
    ensure_dev();
    std::vector<std::deque<Slot*>> mine(b_);
    std::vector<Slot*> ready;
    int64_t pending = 0;
    while (true) {
      if (pending == 0 || poll_new_.load(std::memory_order_acquire)) {
        std::unique_lock<std::mutex> lk(poll_mu_);
        if (pending == 0) {
          poll_idle_ = true;
          poll_cv_.wait(lk, [&] {
            if (poll_stop_) return true;
            for (auto& v : poll_in_)
              if (!v.empty()) return true;
            return false;
          });
          poll_idle_ = false;
        }
        for (int w = 0; w < b_; ++w) {
          for (Slot* sl : poll_in_[w]) mine[w].push_back(sl);
          pending += (int64_t)poll_in_[w].size();
          poll_in_[w].clear();
        }
        poll_new_.store(false, std::memory_order_relaxed);
        if (poll_stop_ && pending == 0) return;
      }
      ready.clear();
      for (int w = 0; w < b_; ++w) {
        auto& q = mine[w];
        while (!q.empty() && job_done(q.front())) {
          ready.push_back(q.front());
          q.pop_front();
          --pending;
        }
      }
      for (Slot* sl : ready) host_cb(&sl->cb);
      if (ready.empty()) {
        if (flag_mode_) {
          for (int k = 0; k < 64; ++k) __builtin_ia32_pause();
        } else {
          std::this_thread::yield();
        }
      }
    }
  }

  // Completion threads of SET_CB_EVENT_BLOCKING, one per worker: the
  // worker's launched jobs in launch order, each waited for by a blocking
  // event synchronisation (the thread sleeps until the runtime signals the
  // event), then released.  A failed wait completes the job with SET_EDEVICE.
  void wait_loop(int w) {
    ensure_dev();
    Waiter& wt = *waiters_[w];
    while (true) {
      Slot* sl = nullptr;
      {
        std::unique_lock<std::mutex> lk(wt.mu);
        wt.cv.wait(lk, [&] { return wt.stop || !wt.q.empty(); });
        if (wt.q.empty()) return;  // stopping, nothing in flight
        sl = wt.q.front();
        wt.q.pop_front();
      }
      const hipError_t e = hipEventSynchronize(sl->ev);
      const CbCtx c = sl->cb;
      c.done(c.ctx, c.job, e == hipSuccess ? SET_OK : SET_EDEVICE);
    }
  }

  void setup_slot(Pipe& p, Slot& sl, const float taps[3]) {
    const SlotLayout& L = p.L;
    char* b = sl.base;
    SlotConst sc;
    sc.hdr = reinterpret_cast<DevSlotHdr*>(b + L.hdr);
    sc.tail = reinterpret_cast<const uint64_t*>(b + L.tail);
    sc.outh = reinterpret_cast<set_out_header*>(b + L.out);
    sc.canary_head = canary_value(sl.tmpl, sl.w, sl.s, 0);
    sc.canary_tail = canary_value(sl.tmpl, sl.w, sl.s, 1);
    const set_job_template& t = p.t;
    const int h = (int)t.height, w = (int)t.width;
    const int64_t npix = (int64_t)h * w;
    auto stage = [&](const void* f, dim3 g, void* args, unsigned blk = kBlock) {
      sl.func[sl.nstages] = f;
      sl.grid[sl.nstages] = g;
      sl.block[sl.nstages] = blk;
      sl.argv[sl.nstages][0] = args;
      ++sl.nstages;
    };
    sl.nstages = 0;
    switch (t.pipeline) {
      case SET_PIPE_BOX_HIST_U8: {
        const unsigned hb = hist_blocks(npix);
        sl.box = BoxArgs{(const uint8_t*)(b + L.in), (uint16_t*)(b + L.b1), h, w, sc.hdr, JobScalars{}};
        sl.div = Div9Args{(const uint16_t*)(b + L.b1), (uint8_t*)(b + L.b2), npix};
        sl.hist = HistArgs{(const uint8_t*)(b + L.b2), npix, (uint32_t*)(b + L.scratch)};
        sl.histf = HistFinalArgs{(const uint32_t*)(b + L.scratch), hb, (uint32_t*)(b + L.out + 64), sc};
        stage((const void*)&k_box3_u8_u16, to_dim3(box_grid(h, w)), &sl.box);
        stage((const void*)&k_div9_u16_u8, dim3(div9_blocks(npix)), &sl.div);
        stage((const void*)&k_hist256_u8, dim3(hb), &sl.hist);
        stage((const void*)&k_hist256_final, dim3(1), &sl.histf);
        break;
      }
      case SET_PIPE_GAUSS_SOBEL_F32: {
        sl.gauss = GaussArgs{(const float*)(b + L.in), (float*)(b + L.b1), h, w, taps[0], taps[1], taps[2], sc.hdr,
                             JobScalars{}};
        const Grid3 sg = sobel_grid(h, w);
        const unsigned nb = (unsigned)sobel_partials(h, w);
        const uint64_t q = ((uint64_t)nb * 4 + 255) / 256 * 256;
        sl.sobel = SobelArgs{(const float*)(b + L.b1), (uint8_t*)(b + L.b2), h, w,
                             t.threshold != 0.f ? t.threshold : 1.0f, (uint32_t*)(b + L.scratch),
                             (float*)(b + L.scratch + q)};
        sl.sobelf = SobelFinalArgs{(const uint32_t*)(b + L.scratch), (const float*)(b + L.scratch + q), nb,
                                   (uint32_t*)(b + L.out + 64), (float*)(b + L.out + 68), sc};
        const bool win = image_window_path(w), full = window_full_width(w);
        const int gr = gauss_win_rows(h, w), sr = sobel_win_rows(h, w);
        // window kernels by rows per wave (2 or 4) and full-width variant
        const void* gks[2][2] = {{(const void*)&k_gauss5_win_f32<2, false>, (const void*)&k_gauss5_win_f32<2, true>},
                                 {(const void*)&k_gauss5_win_f32<4, false>, (const void*)&k_gauss5_win_f32<4, true>}};
        const void* sks[2][2] = {
            {(const void*)&k_sobel_thresh_win_f32<2, false>, (const void*)&k_sobel_thresh_win_f32<2, true>},
            {(const void*)&k_sobel_thresh_win_f32<4, false>, (const void*)&k_sobel_thresh_win_f32<4, true>}};
        const void* gk = win ? gks[gr == 2 ? 0 : 1][full ? 1 : 0] : (const void*)&k_gauss5_f32;
        if (gauss_band_path(w))
          stage(gauss_band_rows(h, w) == 8 ? (const void*)&k_gauss5_band_f32<8> : (const void*)&k_gauss5_band_f32<4>,
                to_dim3(gauss_grid(h, w)), &sl.gauss, (unsigned)kBandCols / 4);
        else
          stage(gk, to_dim3(gauss_grid(h, w)), &sl.gauss);
        const void* sk = win ? sks[sr == 2 ? 0 : 1][full ? 1 : 0] : (const void*)&k_sobel_thresh_f32;
        stage(sk, to_dim3(sg), &sl.sobel);
        stage((const void*)&k_sobel_final, dim3(1), &sl.sobelf);
        break;
      }
      case SET_PIPE_SAXPY_TANH_SUM_F32: {
        sl.vec = VecArgs{t.dev_x_pool, t.dev_y_pool, (float*)(b + L.scratch), sc.hdr, JobScalars{}};
        sl.vec.js.n = t.max_n;
        sl.vecf = VecFinalArgs{(const float*)(b + L.scratch), (float*)(b + L.out + 64), sc};
        stage((const void*)&k_saxpy_tanh_sum_f32, dim3(vec_blocks(t.max_n)), &sl.vec);
        stage((const void*)&k_vec_final, dim3(1), &sl.vecf);
        break;
      }
      case SET_PIPE_SAXPY_BATCH_F32: {
        const uint64_t q = ((uint64_t)t.tiles_max * 4 + 255) / 256 * 256;
        uint32_t* work = (uint32_t*)(b + L.scratch + q);
        sl.vb = VecBatchArgs{(const uint8_t*)(b + L.in), t.dev_x_pool, t.dev_y_pool, (float*)(b + L.scratch), work,
                             sc.hdr, JobScalars{}};
        sl.vbf = VecBatchFinalArgs{(const uint8_t*)(b + L.in), (const float*)(b + L.scratch), work,
                                   (float*)(b + L.out + 64), sc};
        const int vbb = vec_batch_block(t);
        const void* vbk = vbb == 128   ? (const void*)&k_vec_batch_tiles<128>
                          : vbb == 512 ? (const void*)&k_vec_batch_tiles<512>
                          : vbb == 1024 ? (const void*)&k_vec_batch_tiles<1024>
                                        : (const void*)&k_vec_batch_tiles<256>;
        stage(vbk, dim3(t.grid > 0 ? (unsigned)t.grid : (unsigned)kVecBatchGrid), &sl.vb, (unsigned)vbb);
        stage((const void*)&k_vec_batch_final, dim3((t.batch_max + kBlock - 1) / kBlock), &sl.vbf);
        break;
      }
      case SET_PIPE_HOTSPOT_F32: {
        // step k reads T_k and writes T_{k+1}: T_0 is the input, the last
        // step writes the output payload, the others alternate b1 / b2
        const int K = (int)t.max_n;
        const float* P = (const float*)(b + L.in) + (size_t)h * w;
        const void* hk = !image_window_path(w)  ? (const void*)&k_hotspot_f32
                         : window_full_width(w) ? (const void*)&k_hotspot_win_f32<true>
                                                : (const void*)&k_hotspot_win_f32<false>;
        for (int k = 0; k < K; ++k) {
          const float* src = (k == 0) ? (const float*)(b + L.in) : sl.hot[k - 1].tout;
          float* dst = (k == K - 1) ? (float*)(b + L.out + 64) : (float*)(b + ((k % 2 == 0) ? L.b1 : L.b2));
          sl.hot[k] = HotspotArgs{src, P, dst, h, w, k == 0 ? 1 : 0, sc.hdr, JobScalars{}};
          const int hr = hotspot_band_rows(h, w);
          if (hr)
            stage(hr == 16 ? (const void*)&k_hotspot_band_f32<16> : (const void*)&k_hotspot_band_f32<8>,
                  to_dim3(hotspot_grid(h, w)), &sl.hot[k], (unsigned)kBandCols / 4);
          else
            stage(hk, to_dim3(hotspot_grid(h, w)), &sl.hot[k]);
        }
        sl.je = JobEndArgs{sc};
        stage((const void*)&k_job_end, dim3(1), &sl.je);
        break;
      }
      case SET_PIPE_SCAN_LIB_I32_I64:
        sl.jb = JobBeginArgs{sc.hdr, JobScalars{}};
        sl.je = JobEndArgs{sc};
        stage((const void*)&k_job_begin, dim3(1), &sl.jb);
        stage((const void*)&k_job_end, dim3(1), &sl.je);
        break;
      case SET_PIPE_SCAN_I32_I64: {
        const unsigned T = scan_tiles(t.max_n);
        const uint64_t q8 = ((uint64_t)T * 8 + 255) / 256 * 256;
        char* sb = b + L.scratch;
        sl.scan_r = ScanReduceArgs{(const int32_t*)(b + L.in), (int64_t*)sb, T, sc.hdr, JobScalars{}};
        sl.scan_r.js.n = t.max_n;
        sl.scan_s = ScanSpineArgs{(const int64_t*)sb, (int64_t*)(sb + q8), sc, t.max_n};
        sl.scan_d = ScanDownArgs{(const int32_t*)(b + L.in), (const int64_t*)(sb + q8), (void*)(b + L.out + 64),
                                 (t.flags & SET_TF_SCAN_LOW32) ? 1 : 0, t.max_n};
        stage((const void*)&k_scan_reduce_i32, dim3(T), &sl.scan_r);
        stage((const void*)&k_scan_spine_i64, dim3(1), &sl.scan_s);
        stage((const void*)&k_scan_down_i32_i64, dim3(T), &sl.scan_d);
        break;
      }
    }
    // Memory-safety stress: the poisoned range runs from the first buffer
    // after the header to the tail canary (both 256-byte aligned).
    // The batched-vector work counter is the one word kept as zero.
    const uint64_t zero_word = t.pipeline == SET_PIPE_SAXPY_BATCH_F32
                                   ? (uint64_t)(reinterpret_cast<char*>(sl.vb.work) - (b + L.in)) / 4
                                   : ~0ull;
    sl.poison = PoisonArgs{b + L.in, (L.tail - L.in) / 16, zero_word};
    const uint64_t us = t.stress_delay_us;
    sl.delay = DelayArgs{us * clock_khz_ / 1000, 8 * us + 64};
  }

  static bool poisons(const Pipe& p) { return (p.t.flags & SET_TF_POISON) != 0; }
  static bool delays(const Pipe& p) { return p.t.stress_delay_us > 0; }
  static unsigned poison_blocks(const Pipe& p) {
    const uint64_t nvec = (p.L.tail - p.L.in) / 16;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(1024, (nvec + kBlock - 1) / kBlock));
  }
  hipKernelNodeParams stress_params(Pipe& p, Slot& sl, bool poison) {
    hipKernelNodeParams kp{};
    kp.func = poison ? (void*)&k_poison : (void*)&k_stress_delay;
    kp.gridDim = dim3(poison ? poison_blocks(p) : 1);
    kp.blockDim = dim3(poison ? kBlock : 64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = poison ? sl.poison_argv : sl.delay_argv;
    kp.extra = nullptr;
    return kp;
  }
  hipError_t launch_stress(Pipe& p, Slot& sl, bool poison, hipStream_t st) {
    const hipKernelNodeParams kp = stress_params(p, sl, poison);
    return hipLaunchKernel(kp.func, kp.gridDim, kp.blockDim, kp.kernelParams, 0, st);
  }

  // Write the job's scalars into the slot's first-stage argument block and
  // record its host endpoints.
  void set_scalars(Pipe& p, Slot& sl, const JobRec* j) {
    JobScalars js{};
    js.job_id = j->id;
    js.seq = j->seq;
    js.user_tag = j->args.user_tag;
    js.n = j->args.n;
    js.x_off = j->args.x_off;
    js.y_off = j->args.y_off;
    js.worker = (uint32_t)j->worker;
    js.slot = (uint32_t)j->slot;
    js.a = j->args.a;
    switch (p.t.pipeline) {
      case SET_PIPE_BOX_HIST_U8:
        sl.box.js = js;
        break;
      case SET_PIPE_GAUSS_SOBEL_F32:
        sl.gauss.js = js;
        break;
      case SET_PIPE_SAXPY_TANH_SUM_F32:
        sl.vec.js = js;
        sl.grid[0] = dim3(vec_blocks(js.n));
        break;
      case SET_PIPE_SCAN_I32_I64:
        if (js.n == 0) js.n = p.t.max_n;
        sl.scan_r.js = js;
        sl.scan_s.n = js.n;
        sl.scan_d.n = js.n;
        break;
      case SET_PIPE_SCAN_LIB_I32_I64:
        js.n = p.t.max_n;
        sl.jb.js = js;
        break;
      case SET_PIPE_HOTSPOT_F32:
        sl.hot[0].js = js;
        break;
      case SET_PIPE_SAXPY_BATCH_F32:
        sl.vb.js = js;
        sl.grid[0] = dim3(j->args.grid ? j->args.grid : (p.t.grid > 0 ? (unsigned)p.t.grid : (unsigned)kVecBatchGrid));
        break;
    }
    sl.host_in = j->args.host_in;
    sl.in_bytes = pipeline_in_bytes(p.t, js.n);
    sl.host_out = j->args.host_out;
    sl.out_bytes = pipeline_out_bytes(p.t, js.n);
  }

  hipKernelNodeParams kparams(Slot& sl, int i) {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(sl.func[i]);
    kp.gridDim = sl.grid[i];
    kp.blockDim = dim3(sl.block[i]);
    kp.sharedMemBytes = 0;
    kp.kernelParams = sl.argv[i];
    kp.extra = nullptr;
    return kp;
  }

  hipKernelNodeParams copy_params(void** argv, bool to_device, unsigned blocks = kCopyBlocks) {
    hipKernelNodeParams kp{};
    kp.func = to_device ? (void*)&k_copy_in : (void*)&k_copy_out;
    kp.gridDim = dim3(blocks);
    kp.blockDim = dim3(kBlock);
    kp.sharedMemBytes = 0;
    kp.kernelParams = argv;
    kp.extra = nullptr;
    return kp;
  }

  // The library stage of a library-call template (no-op for the others).
  hipError_t library_stage(Pipe& p, Slot& sl, hipStream_t st) {
    if (!lib_template(p.t)) return hipSuccess;
    size_t bytes = sl.lib_ws_bytes;
    return lib_scan(sl.lib_ws, bytes, reinterpret_cast<const int32_t*>(sl.base + p.L.in),
                    reinterpret_cast<int64_t*>(sl.base + p.L.out + 64), (size_t)p.t.max_n, st);
  }

  // SET_COPY_ASYNC_IN: the job's input copy, ordered ahead of its graph on
  // stream st.  If bind already issued it (SET mode with input-copy
  // streams), st only waits on its event.  Otherwise, without input-copy
  // streams (and for a stolen job in SET mode) it runs on st itself; in the
  // other modes with input-copy streams it runs on input-copy stream w % C
  // and st waits on its event, so at most C DMA copies are in flight.  The
  // slot was released before this job was bound to it, so the copy cannot
  // overwrite an input that a running graph still reads.
  hipError_t input_ahead(Pipe& p, Slot& sl, hipStream_t st, int w) {
    if (!in_ahead(p.t) || sl.in_bytes == 0) return hipSuccess;
    if (sl.in_prefetched) {
      sl.in_prefetched = false;
      return hipStreamWaitEvent(st, sl.in_ev, 0);
    }
    if (sl.in_stale) {
      sl.in_stale = false;
      const hipError_t e = hipStreamWaitEvent(st, sl.in_ev, 0);
      if (e != hipSuccess) return e;
    }
    if (copy_streams_.empty() || !sl.in_ev || cfg_.mode == SET_MODE_SET)
      return hipMemcpyAsync(sl.base + p.L.in, sl.host_in, sl.in_bytes, hipMemcpyHostToDevice, st);
    hipStream_t cs = copy_streams_[(size_t)w % copy_streams_.size()];
    hipError_t e = hipMemcpyAsync(sl.base + p.L.in, sl.host_in, sl.in_bytes, hipMemcpyHostToDevice, cs);
    if (e == hipSuccess) e = hipEventRecord(sl.in_ev, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, sl.in_ev, 0);
    return e;
  }

  int add_chain(Pipe& p, Slot& sl, hipGraph_t g, ChainNodes* cn, std::string* err) {
    if (lib_template(p.t)) {
      if (err) *err = "library-call templates are built by stream capture only";
      return SET_EUNSUPPORTED;
    }
    const bool kcopy = in_by_kernel(p.t);
    hipGraphNode_t prev = nullptr;
    if (p.L.in_cap > 0 && !in_ahead(p.t)) {
      if (kcopy) {
        sl.h2d_copy = CopyArgs{p.placeholder, sl.base + p.L.in, p.L.in_cap};
        hipKernelNodeParams kp = copy_params(sl.h2d_argv, true);
        HIPCK(hipGraphAddKernelNode(&cn->h2d, g, nullptr, 0, &kp));
      } else {
        HIPCK(hipGraphAddMemcpyNode1D(&cn->h2d, g, nullptr, 0, sl.base + p.L.in, p.placeholder, p.L.in_cap,
                                      hipMemcpyHostToDevice));
      }
      prev = cn->h2d;
    }
    if (delays(p)) {
      hipKernelNodeParams kp = stress_params(p, sl, false);
      HIPCK(hipGraphAddKernelNode(&cn->delay, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
      prev = cn->delay;
    }
    for (int i = 0; i < sl.nstages; ++i) {
      hipKernelNodeParams kp = kparams(sl, i);
      HIPCK(hipGraphAddKernelNode(&cn->k[i], g, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
      prev = cn->k[i];
    }
    if (out_by_kernel(p.t)) {
      sl.d2h_copy = CopyArgs{sl.base + p.L.out, p.placeholder, p.L.out_cap};
      hipKernelNodeParams kp = copy_params(sl.d2h_argv, false, d2h_copy_blocks(p.L.out_cap));
      HIPCK(hipGraphAddKernelNode(&cn->d2h, g, &prev, 1, &kp));
    } else {
      HIPCK(hipGraphAddMemcpyNode1D(&cn->d2h, g, &prev, 1, p.placeholder, sl.base + p.L.out, p.L.out_cap,
                                    hipMemcpyDeviceToHost));
    }
    prev = cn->d2h;
    if (poisons(p)) {
      hipKernelNodeParams kp = stress_params(p, sl, true);
      HIPCK(hipGraphAddKernelNode(&cn->poison, g, &prev, 1, &kp));
      prev = cn->poison;
    }
    if (p.words && g == sl.graph) {
      hipKernelNodeParams kf = flag_params(sl);
      HIPCK(hipGraphAddKernelNode(&cn->flag, g, &prev, 1, &kf));
    }
    return SET_OK;
  }

  hipKernelNodeParams flag_params(Slot& sl) {
    hipKernelNodeParams kp{};
    kp.func = (void*)&k_done_flag;
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = sl.flag_argv;
    kp.extra = nullptr;
    return kp;
  }

  // Stream capture of the job's launch sequence (the copies bound to the
  // placeholder), then the captured chain is walked from its root to find
  // the nodes the binder updates.
  int capture_chain(Pipe& p, Slot& sl, hipStream_t st, hipGraph_t* out, ChainNodes* cn, std::string* err) {
    const bool kcopy = in_by_kernel(p.t);
    const bool in_node = p.L.in_cap > 0 && !in_ahead(p.t);
    HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    if (in_node) {
      if (kcopy) {
        sl.h2d_copy = CopyArgs{p.placeholder, sl.base + p.L.in, p.L.in_cap};
        HIPCK(hipLaunchKernel((const void*)&k_copy_in, dim3(kCopyBlocks), dim3(kBlock), sl.h2d_argv, 0, st));
      } else {
        HIPCK(hipMemcpyAsync(sl.base + p.L.in, p.placeholder, p.L.in_cap, hipMemcpyHostToDevice, st));
      }
    }
    if (delays(p)) HIPCK(launch_stress(p, sl, false, st));
    for (int i = 0; i < sl.nstages; ++i) {
      if (i == 1) HIPCK(library_stage(p, sl, st));
      HIPCK(hipLaunchKernel(sl.func[i], sl.grid[i], dim3(sl.block[i]), sl.argv[i], 0, st));
    }
    if (out_by_kernel(p.t)) {
      sl.d2h_copy = CopyArgs{sl.base + p.L.out, p.placeholder, p.L.out_cap};
      HIPCK(hipLaunchKernel((const void*)&k_copy_out, dim3(d2h_copy_blocks(p.L.out_cap)), dim3(kBlock), sl.d2h_argv, 0, st));
    } else {
      HIPCK(hipMemcpyAsync(p.placeholder, sl.base + p.L.out, p.L.out_cap, hipMemcpyDeviceToHost, st));
    }
    if (poisons(p)) HIPCK(launch_stress(p, sl, true, st));
    if (p.words) HIPCK(hipLaunchKernel((const void*)&k_done_flag, dim3(1), dim3(64), sl.flag_argv, 0, st));
    HIPCK(hipStreamEndCapture(st, out));
    size_t n = 0;
    HIPCK(hipGraphGetNodes(*out, nullptr, &n));
    std::vector<hipGraphNode_t> nodes(n);
    HIPCK(hipGraphGetNodes(*out, nodes.data(), &n));
    const size_t fixed =
        (in_node ? 1 : 0) + (delays(p) ? 1 : 0) + sl.nstages + 1 + (poisons(p) ? 1 : 0) + (p.words ? 1 : 0);
    const size_t lib_nodes = n - std::min(n, fixed);  // captured library kernels between stages 0 and 1
    if (n < fixed || (lib_template(p.t) ? lib_nodes < 1 : lib_nodes != 0)) {
      if (err) *err = "captured graph has an unexpected number of nodes";
      return SET_EDEVICE;
    }
    // order the linear chain: start at the node with no dependencies
    std::vector<hipGraphNode_t> order;
    hipGraphNode_t cur = nullptr;
    for (hipGraphNode_t nd : nodes) {
      size_t deps = 0;
      HIPCK(hipGraphNodeGetDependencies(nd, nullptr, &deps));
      if (deps == 0) cur = nd;
    }
    while (cur && order.size() < n) {
      order.push_back(cur);
      size_t nd = 0;
      HIPCK(hipGraphNodeGetDependentNodes(cur, nullptr, &nd));
      if (nd == 0) break;
      if (nd != 1) {
        if (err) *err = "captured graph is not a chain";
        return SET_EDEVICE;
      }
      HIPCK(hipGraphNodeGetDependentNodes(cur, &cur, &nd));
    }
    if (order.size() != n) {
      if (err) *err = "captured graph is not a chain";
      return SET_EDEVICE;
    }
    size_t k = 0;
    if (in_node) cn->h2d = order[k++];
    if (delays(p)) cn->delay = order[k++];
    for (int i = 0; i < sl.nstages; ++i) {
      if (i == 1) {
        // the library's nodes: kernels only (no memset or memcpy nodes in a replayed graph)
        for (size_t m = 0; m < lib_nodes; ++m) {
          hipGraphNodeType ty;
          HIPCK(hipGraphNodeGetType(order[k + m], &ty));
          if (ty != hipGraphNodeTypeKernel) {
            if (err) *err = "captured library call recorded a node that is not a kernel";
            return SET_EUNSUPPORTED;
          }
        }
        k += lib_nodes;
      }
      hipKernelNodeParams kp{};
      HIPCK(hipGraphKernelNodeGetParams(order[k], &kp));
      if (kp.func != sl.func[i]) {
        if (err) *err = "captured stage order differs from the template";
        return SET_EDEVICE;
      }
      cn->k[i] = order[k++];
    }
    cn->d2h = order[k++];
    if (poisons(p)) cn->poison = order[k++];
    if (p.words) cn->flag = order[k];
    return SET_OK;
  }

  // UpdateGraphParams: retarget an executable's chain to the slot's current
  // binding (H2D source, first kernel's argument block and grid, D2H target).
  int update_exec(Pipe& p, Slot& sl, hipGraphExec_t ex, const ChainNodes& cn, std::string* err) {
    const bool kcopy = in_by_kernel(p.t);
    if (sl.in_bytes && cn.h2d) {
      if (kcopy) {
        sl.h2d_copy = CopyArgs{sl.host_in, sl.base + p.L.in, sl.in_bytes};
        hipKernelNodeParams kp = copy_params(sl.h2d_argv, true);
        HIPCK(hipGraphExecKernelNodeSetParams(ex, cn.h2d, &kp));
      } else {
        HIPCK(hipGraphExecMemcpyNodeSetParams1D(ex, cn.h2d, sl.base + p.L.in, sl.host_in, sl.in_bytes,
                                                hipMemcpyHostToDevice));
      }
    }
    hipKernelNodeParams kp = kparams(sl, 0);
    HIPCK(hipGraphExecKernelNodeSetParams(ex, cn.k[0], &kp));
    if (p.t.pipeline == SET_PIPE_SCAN_I32_I64) {  // the spine and the downsweep carry n too
      for (int i = 1; i <= 2; ++i) {
        hipKernelNodeParams kd = kparams(sl, i);
        HIPCK(hipGraphExecKernelNodeSetParams(ex, cn.k[i], &kd));
      }
    }
    if (out_by_kernel(p.t)) {
      sl.d2h_copy = CopyArgs{sl.base + p.L.out, sl.host_out, sl.out_bytes};
      hipKernelNodeParams kd = copy_params(sl.d2h_argv, false, d2h_copy_blocks(p.L.out_cap));
      HIPCK(hipGraphExecKernelNodeSetParams(ex, cn.d2h, &kd));
    } else {
      HIPCK(hipGraphExecMemcpyNodeSetParams1D(ex, cn.d2h, sl.host_out, sl.base + p.L.out, sl.out_bytes,
                                              hipMemcpyDeviceToHost));
    }
    return SET_OK;
  }

  set_config cfg_{};
  int b_ = 0, d_ = 0, dev_ = -1;
  bool own_streams_ = false, down_ = false;
  std::vector<hipStream_t> streams_, cb_streams_;
  std::unique_ptr<std::mutex[]> cb_mu_;  // one per callback stream
  std::vector<hipStream_t> copy_streams_;  // input-copy streams (set_config.input_copy_streams)
  hipStream_t define_stream_ = nullptr;    // template capture and graph upload, never a worker's
  std::vector<std::unique_ptr<Pipe>> pipes_;
  std::atomic<uint64_t> sync_ns_{0};
  // event polling
  struct Waiter {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Slot*> q;
    bool stop = false;
  };
  std::vector<std::unique_ptr<Waiter>> waiters_;  // SET_CB_EVENT_BLOCKING
  bool blocking_ = false;
  std::thread poller_;
  std::mutex poll_mu_;
  std::condition_variable poll_cv_;
  std::vector<std::vector<Slot*>> poll_in_;  // launched, not yet taken over by the completion thread
  bool poll_idle_ = false;                     // completion thread waits on poll_cv_
  std::atomic<bool> poll_new_{false};          // poll_in_ holds entries
  bool poll_stop_ = false;
  bool flag_mode_ = false;
  uint64_t clock_khz_ = 100000;  // rate of the device's constant clock (stress delay)
};

}  // namespace

Backend* make_hip_backend() { return new HipBackend(); }

}  // namespace setrt
