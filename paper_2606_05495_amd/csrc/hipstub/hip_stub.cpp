// Host-only HIP runtime stand-in and host versions of the stage kernels, for
// the ThreadSanitizer build of the HIP backend (see hip/hip_runtime.h here).
#include "hip/hip_runtime.h"

#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"

// ------------------------------------------------------------------ kernel registry
namespace hipstub {
namespace {
struct Kernel {
  size_t bytes;
  Invoke run;
};
std::unordered_map<const void*, Kernel>& registry() {
  static std::unordered_map<const void*, Kernel> r;
  return r;
}
std::atomic<uint64_t> g_launches{0}, g_hazards{0}, g_walk{0};
}  // namespace
void register_kernel(const void* func, size_t arg_bytes, Invoke run) { registry()[func] = Kernel{arg_bytes, run}; }
uint64_t launches() { return g_launches.load(); }
uint64_t updates_while_in_flight() { return g_hazards.load(); }
const Kernel* find_kernel(const void* f) {
  auto it = registry().find(f);
  return it == registry().end() ? nullptr : &it->second;
}
}  // namespace hipstub

// ------------------------------------------------------------------ runtime objects
struct hipGraphNode {
  hipGraphNodeType type = hipGraphNodeTypeKernel;
  const void* func = nullptr;
  dim3 grid, block;
  std::vector<char> args;
  void* dst = nullptr;
  const void* src = nullptr;
  size_t bytes = 0;
  std::vector<hipGraphNode*> deps, dependents;
};

struct ihipGraph {
  std::vector<hipGraphNode*> nodes;
  ~ihipGraph() {
    for (hipGraphNode* n : nodes) delete n;
  }
  hipGraphNode* add(const hipGraphNode_t* deps, size_t ndeps) {
    hipGraphNode* n = new hipGraphNode();
    for (size_t i = 0; i < ndeps; ++i) {
      n->deps.push_back(deps[i]);
      deps[i]->dependents.push_back(n);
    }
    nodes.push_back(n);
    return n;
  }
};

struct ExecNode {
  hipGraphNodeType type;
  const void* func;
  std::vector<char> args;  // the executable's own copy, read when the node runs
  void* dst;
  const void* src;
  size_t bytes;
};

struct hipGraphExec {
  std::vector<ExecNode> nodes;  // insertion order is a topological order for every graph built here
  std::unordered_map<const hipGraphNode*, size_t> index;
  std::atomic<int> queued{0};   // launches enqueued and not yet started
  std::atomic<int> pos{-1};     // node the running launch is at (-1: none)
};

struct ihipEvent_t {
  std::mutex mu;
  std::condition_variable cv;
  uint64_t recorded = 0, completed = 0;
};

struct ihipStream_t {
  std::mutex mu;
  std::condition_variable cv, idle;
  std::deque<std::function<void()>> q;
  bool busy = false, stop = false;
  std::thread th;
  ihipGraph* cap = nullptr;  // graph being captured, if any
  hipGraphNode* cap_last = nullptr;
  std::thread::id cap_thread;
};

namespace {
std::mutex g_streams_mu;
std::vector<ihipStream_t*> g_streams;

void stream_loop(ihipStream_t* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv.wait(lk, [&] { return s->stop || !s->q.empty(); });
    if (s->q.empty()) return;
    std::function<void()> op = std::move(s->q.front());
    s->q.pop_front();
    s->busy = true;
    lk.unlock();
    op();
    lk.lock();
    s->busy = false;
    if (s->q.empty()) s->idle.notify_all();
  }
}

void enqueue(ihipStream_t* s, std::function<void()> op) {
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->q.push_back(std::move(op));
  }
  s->cv.notify_one();
}

// A call that would enqueue onto a stream another thread is capturing: the
// real runtime would record it into that thread's graph.  Refused here so a
// stress run shows it.
bool foreign_capture(ihipStream_t* s) { return s->cap && s->cap_thread != std::this_thread::get_id(); }

void run_exec(hipGraphExec* ex) {
  ex->queued.fetch_sub(1);
  const size_t n = ex->nodes.size();
  for (size_t i = 0; i < n; ++i) {
    ex->pos.store((int)i);
    const ExecNode& en = ex->nodes[i];
    if (en.type == hipGraphNodeTypeKernel) {
      const hipstub::Kernel* k = hipstub::find_kernel(en.func);
      k->run(en.func, en.args.data());
    } else {
      std::memcpy(en.dst, en.src, en.bytes);
    }
  }
  ex->pos.store(-1);
}

void note_update(hipGraphExec* ex, size_t idx) {
  const int p = ex->pos.load();
  if (ex->queued.load() > 0 || (p >= 0 && (size_t)p <= idx)) hipstub::g_hazards.fetch_add(1);
}
}  // namespace

// ------------------------------------------------------------------ device, memory
const char* hipGetErrorString(hipError_t e) {
  switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorInvalidValue: return "hipErrorInvalidValue (stub)";
    case hipErrorNotReady: return "hipErrorNotReady";
    case hipErrorNotSupported: return "hipErrorNotSupported (stub)";
    default: return "hipErrorUnknown (stub)";
  }
}
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t attr, int dev) {
  if (dev != 0 || attr != hipDeviceAttributeWallClockRate) return hipErrorInvalidValue;
  *value = 100000;  // kHz
  return hipSuccess;
}
hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
  std::vector<ihipStream_t*> all;
  {
    std::lock_guard<std::mutex> g(g_streams_mu);
    all = g_streams;
  }
  for (ihipStream_t* s : all) hipStreamSynchronize(s);
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t bytes) {
  *p = std::aligned_alloc(256, (bytes + 255) / 256 * 256 + 256);
  return *p ? hipSuccess : hipErrorUnknown;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemset(void* dst, int value, size_t bytes) {
  std::memset(dst, value, bytes);
  return hipSuccess;
}

// ------------------------------------------------------------------ streams
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  ihipStream_t* st = new ihipStream_t();
  st->th = std::thread(stream_loop, st);
  {
    std::lock_guard<std::mutex> g(g_streams_mu);
    g_streams.push_back(st);
  }
  *s = st;
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  {
    std::lock_guard<std::mutex> g(g_streams_mu);
    for (size_t i = 0; i < g_streams.size(); ++i)
      if (g_streams[i] == s) {
        g_streams.erase(g_streams.begin() + i);
        break;
      }
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  s->th.join();
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  std::unique_lock<std::mutex> lk(s->mu);
  s->idle.wait(lk, [&] { return s->q.empty() && !s->busy; });
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
  if (foreign_capture(s)) return hipErrorUnknown;
  if (s->cap) {
    hipGraphNode* n = s->cap->add(s->cap_last ? &s->cap_last : nullptr, s->cap_last ? 1 : 0);
    n->type = hipGraphNodeTypeMemcpy;
    n->dst = dst;
    n->src = src;
    n->bytes = bytes;
    s->cap_last = n;
    return hipSuccess;
  }
  (void)kind;
  enqueue(s, [=] { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipLaunchKernel(const void* func, dim3 grid, dim3 block, void** args, size_t, hipStream_t s) {
  const hipstub::Kernel* k = hipstub::find_kernel(func);
  if (!k || !args || !args[0]) return hipErrorInvalidValue;
  if (foreign_capture(s)) return hipErrorUnknown;
  std::vector<char> bytes((const char*)args[0], (const char*)args[0] + k->bytes);  // copied at launch
  if (s->cap) {
    hipGraphNode* n = s->cap->add(s->cap_last ? &s->cap_last : nullptr, s->cap_last ? 1 : 0);
    n->type = hipGraphNodeTypeKernel;
    n->func = func;
    n->grid = grid;
    n->block = block;
    n->args = std::move(bytes);
    s->cap_last = n;
    return hipSuccess;
  }
  hipstub::g_launches.fetch_add(1);
  enqueue(s, [func, k, bytes = std::move(bytes)] { k->run(func, bytes.data()); });
  return hipSuccess;
}
hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void* user) {
  if (s->cap) return hipErrorNotSupported;
  enqueue(s, [=] { fn(user); });
  return hipSuccess;
}

// ------------------------------------------------------------------ events
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (s->cap) return hipErrorNotSupported;
  uint64_t g;
  {
    std::lock_guard<std::mutex> l(e->mu);
    g = ++e->recorded;
  }
  enqueue(s, [e, g] {
    {
      std::lock_guard<std::mutex> l(e->mu);
      if (e->completed < g) e->completed = g;
    }
    e->cv.notify_all();
  });
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::mutex> l(e->mu);
  return e->completed >= e->recorded ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::unique_lock<std::mutex> l(e->mu);
  const uint64_t g = e->recorded;
  e->cv.wait(l, [&] { return e->completed >= g; });
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  if (s->cap) return hipErrorNotSupported;
  uint64_t g;
  {
    std::lock_guard<std::mutex> l(e->mu);
    g = e->recorded;
  }
  enqueue(s, [e, g] {
    std::unique_lock<std::mutex> l(e->mu);
    e->cv.wait(l, [&] { return e->completed >= g; });
  });
  return hipSuccess;
}

// ------------------------------------------------------------------ graphs
hipError_t hipGraphCreate(hipGraph_t* g, unsigned) {
  *g = new ihipGraph();
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphAddKernelNode(hipGraphNode_t* node, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                 const hipKernelNodeParams* p) {
  const hipstub::Kernel* k = hipstub::find_kernel(p->func);
  if (!k || !p->kernelParams || !p->kernelParams[0]) return hipErrorInvalidValue;
  hipGraphNode* n = g->add(deps, ndeps);
  n->type = hipGraphNodeTypeKernel;
  n->func = p->func;
  n->grid = p->gridDim;
  n->block = p->blockDim;
  n->args.assign((const char*)p->kernelParams[0], (const char*)p->kernelParams[0] + k->bytes);
  *node = n;
  return hipSuccess;
}
hipError_t hipGraphAddMemcpyNode1D(hipGraphNode_t* node, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                   void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  hipGraphNode* n = g->add(deps, ndeps);
  n->type = hipGraphNodeTypeMemcpy;
  n->dst = dst;
  n->src = src;
  n->bytes = bytes;
  *node = n;
  return hipSuccess;
}
template <class V>
static hipError_t list_out(const V& v, hipGraphNode_t* out, size_t* n) {
  if (!out) {
    *n = v.size();
    return hipSuccess;
  }
  const size_t k = std::min(*n, v.size());
  for (size_t i = 0; i < k; ++i) out[i] = v[i];
  *n = k;
  return hipSuccess;
}
hipError_t hipGraphGetNodes(hipGraph_t g, hipGraphNode_t* nodes, size_t* n) { return list_out(g->nodes, nodes, n); }
hipError_t hipGraphNodeGetDependencies(hipGraphNode_t node, hipGraphNode_t* deps, size_t* n) {
  return list_out(node->deps, deps, n);
}
hipError_t hipGraphNodeGetDependentNodes(hipGraphNode_t node, hipGraphNode_t* deps, size_t* n) {
  return list_out(node->dependents, deps, n);
}
hipError_t hipGraphNodeGetType(hipGraphNode_t node, hipGraphNodeType* t) {
  *t = node->type;
  return hipSuccess;
}
hipError_t hipGraphKernelNodeGetParams(hipGraphNode_t node, hipKernelNodeParams* p) {
  if (node->type != hipGraphNodeTypeKernel) return hipErrorInvalidValue;
  p->func = const_cast<void*>(node->func);
  p->gridDim = node->grid;
  p->blockDim = node->block;
  p->kernelParams = nullptr;
  p->extra = nullptr;
  p->sharedMemBytes = 0;
  return hipSuccess;
}
hipError_t hipGraphInstantiateWithFlags(hipGraphExec_t* ex, hipGraph_t g, unsigned long long) {
  hipGraphExec* e = new hipGraphExec();
  for (size_t i = 0; i < g->nodes.size(); ++i) {
    const hipGraphNode* n = g->nodes[i];
    e->nodes.push_back(ExecNode{n->type, n->func, n->args, n->dst, n->src, n->bytes});
    e->index[n] = i;
  }
  *ex = e;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
  delete ex;
  return hipSuccess;
}
hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t ex, hipGraphNode_t node, const hipKernelNodeParams* p) {
  auto it = ex->index.find(node);
  const hipstub::Kernel* k = hipstub::find_kernel(p->func);
  if (it == ex->index.end() || !k || !p->kernelParams || !p->kernelParams[0]) return hipErrorInvalidValue;
  ExecNode& en = ex->nodes[it->second];
  if (en.type != hipGraphNodeTypeKernel || en.args.size() != k->bytes) return hipErrorInvalidValue;
  note_update(ex, it->second);
  en.func = p->func;
  std::memcpy(en.args.data(), p->kernelParams[0], k->bytes);  // in place: a concurrent launch reading it races
  return hipSuccess;
}
hipError_t hipGraphExecMemcpyNodeSetParams1D(hipGraphExec_t ex, hipGraphNode_t node, void* dst, const void* src,
                                             size_t bytes, hipMemcpyKind) {
  auto it = ex->index.find(node);
  if (it == ex->index.end()) return hipErrorInvalidValue;
  ExecNode& en = ex->nodes[it->second];
  if (en.type != hipGraphNodeTypeMemcpy) return hipErrorInvalidValue;
  note_update(ex, it->second);
  en.dst = dst;
  en.src = src;
  en.bytes = bytes;
  return hipSuccess;
}
hipError_t hipGraphUpload(hipGraphExec_t, hipStream_t s) { return s->cap ? hipErrorNotSupported : hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s) {
  if (s->cap) return hipErrorNotSupported;
  if (foreign_capture(s)) return hipErrorUnknown;
  // The launching thread walks the executable's nodes (as the runtime does
  // when it builds the dispatch packets): plain reads of every node's
  // parameters, so an update of this executable on another thread at the
  // same time is a race ThreadSanitizer reports.
  uint64_t sum = 0;
  for (const ExecNode& en : ex->nodes) {
    sum += (uint64_t)(uintptr_t)en.func + (uint64_t)(uintptr_t)en.dst + en.bytes;
    for (char ch : en.args) sum += (unsigned char)ch;
  }
  hipstub::g_walk.fetch_add(sum & 1);
  hipstub::g_launches.fetch_add(1);
  ex->queued.fetch_add(1);
  enqueue(s, [ex] { run_exec(ex); });
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (s->cap) return hipErrorInvalidValue;
  s->cap = new ihipGraph();
  s->cap_last = nullptr;
  s->cap_thread = std::this_thread::get_id();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!s->cap || s->cap_thread != std::this_thread::get_id()) return hipErrorInvalidValue;
  *g = s->cap;
  s->cap = nullptr;
  s->cap_last = nullptr;
  return hipSuccess;
}

// ------------------------------------------------------------------ kernels (host versions)
// Only what the scheduler's correctness shows through: the first stage
// writes the job's scalars into the slot header, the last one checks the
// canaries and publishes the output header, the copy kernels copy, and the
// completion-word kernel stores the binding sequence number with a release.
namespace setrt {
namespace {
void stamp(DevSlotHdr* h, const JobScalars& js) {
  h->job_id = js.job_id;
  h->seq = js.seq;
  h->user_tag = js.user_tag;
  h->worker = js.worker;
  h->slot = js.slot;
  h->n = js.n;
}
void publish(const SlotConst& sc) {
  const DevSlotHdr* h = sc.hdr;
  set_out_header* o = sc.outh;
  const bool canaries = h->canary_head == sc.canary_head && *sc.tail == sc.canary_tail;
  o->job_id = h->job_id;
  o->seq = h->seq;
  o->worker = h->worker;
  o->slot = h->slot;
  o->user_tag = h->user_tag;
  o->canary_ok = canaries ? 1u : 0u;
  o->reserved[0] = o->reserved[1] = o->reserved[2] = 0;
  o->magic = SET_OUT_MAGIC;
}
}  // namespace

void k_copy_in(CopyArgs a) { std::memcpy(a.dst, a.src, a.bytes); }
void k_copy_out(CopyArgs a) { std::memcpy(a.dst, a.src, a.bytes); }
void k_ref_copy(RefCopyArgs a) { std::memcpy(a.dst, a.src, a.nvec * 16); }
void k_done_flag(DoneFlagArgs a) { __atomic_store_n(a.word, a.hdr->seq, __ATOMIC_RELEASE); }
void k_poison(PoisonArgs a) {
  std::memset(a.p, 0xFF, a.nvec * 16);
  if (a.zero_word != ~0ull) reinterpret_cast<uint32_t*>(a.p)[a.zero_word] = 0;
}
void k_stress_delay(DelayArgs a) {  // the stand-in clock runs at 100 MHz
  std::this_thread::sleep_for(std::chrono::nanoseconds(a.ticks * 10));
}
void k_job_begin(JobBeginArgs a) { stamp(a.hdr, a.js); }
void k_job_end(JobEndArgs a) { publish(a.sc); }
template <bool FULL>
void k_hotspot_win_f32(HotspotArgs a) {
  if (a.first) stamp(a.hdr, a.js);
}
template void k_hotspot_win_f32<true>(HotspotArgs);
template void k_hotspot_win_f32<false>(HotspotArgs);
template <int R>
void k_hotspot_band_f32(HotspotArgs a) {
  if (a.first) stamp(a.hdr, a.js);
}
template void k_hotspot_band_f32<8>(HotspotArgs);
template void k_hotspot_band_f32<16>(HotspotArgs);
void k_hotspot_f32(HotspotArgs a) {
  if (a.first) stamp(a.hdr, a.js);
}
void k_box3_u8_u16(BoxArgs a) { stamp(a.hdr, a.js); }
void k_div9_u16_u8(Div9Args) {}
void k_hist256_u8(HistArgs) {}
void k_hist256_final(HistFinalArgs a) { publish(a.sc); }
void k_gauss5_f32(GaussArgs a) { stamp(a.hdr, a.js); }
template <int R, bool FULL>
void k_gauss5_win_f32(GaussArgs a) {
  stamp(a.hdr, a.js);
}
template void k_gauss5_win_f32<2, true>(GaussArgs);
template void k_gauss5_win_f32<2, false>(GaussArgs);
template void k_gauss5_win_f32<4, true>(GaussArgs);
template void k_gauss5_win_f32<4, false>(GaussArgs);
template <int R>
void k_gauss5_band_f32(GaussArgs a) {
  stamp(a.hdr, a.js);
}
template void k_gauss5_band_f32<4>(GaussArgs);
template void k_gauss5_band_f32<8>(GaussArgs);
void k_sobel_thresh_f32(SobelArgs) {}
template <int R, bool FULL>
void k_sobel_thresh_win_f32(SobelArgs) {}
template void k_sobel_thresh_win_f32<2, true>(SobelArgs);
template void k_sobel_thresh_win_f32<2, false>(SobelArgs);
template void k_sobel_thresh_win_f32<4, true>(SobelArgs);
template void k_sobel_thresh_win_f32<4, false>(SobelArgs);
void k_sobel_final(SobelFinalArgs a) { publish(a.sc); }
void k_saxpy_tanh_sum_f32(VecArgs a) { stamp(a.hdr, a.js); }
void k_vec_final(VecFinalArgs a) { publish(a.sc); }
template <int BLOCK>
void k_vec_batch_tiles(VecBatchArgs a) {
  stamp(a.hdr, a.js);
}
template void k_vec_batch_tiles<128>(VecBatchArgs);
template void k_vec_batch_tiles<256>(VecBatchArgs);
template void k_vec_batch_tiles<512>(VecBatchArgs);
template void k_vec_batch_tiles<1024>(VecBatchArgs);
void k_vec_batch_final(VecBatchFinalArgs a) { publish(a.sc); }
void k_scan_reduce_i32(ScanReduceArgs a) { stamp(a.hdr, a.js); }
void k_scan_spine_i64(ScanSpineArgs a) { publish(a.sc); }
void k_scan_down_i32_i64(ScanDownArgs) {}
hipError_t lib_scan(void*, size_t& ws_bytes, const int32_t*, int64_t*, size_t, hipStream_t) {
  ws_bytes = 256;
  return hipErrorNotSupported;
}

namespace {
struct Register {
  Register() {
    using hipstub::register_kernel;
    register_kernel(&k_copy_in);
    register_kernel(&k_copy_out);
    register_kernel(&k_ref_copy);
    register_kernel(&k_done_flag);
    register_kernel(&k_poison);
    register_kernel(&k_stress_delay);
    register_kernel(&k_job_begin);
    register_kernel(&k_job_end);
    register_kernel(&k_hotspot_win_f32<true>);
    register_kernel(&k_hotspot_win_f32<false>);
    register_kernel(&k_hotspot_f32);
    register_kernel(&k_hotspot_band_f32<8>);
    register_kernel(&k_hotspot_band_f32<16>);
    register_kernel(&k_box3_u8_u16);
    register_kernel(&k_div9_u16_u8);
    register_kernel(&k_hist256_u8);
    register_kernel(&k_hist256_final);
    register_kernel(&k_gauss5_f32);
    register_kernel(&k_gauss5_win_f32<2, true>);
    register_kernel(&k_gauss5_win_f32<2, false>);
    register_kernel(&k_gauss5_win_f32<4, true>);
    register_kernel(&k_gauss5_win_f32<4, false>);
    register_kernel(&k_gauss5_band_f32<4>);
    register_kernel(&k_gauss5_band_f32<8>);
    register_kernel(&k_sobel_thresh_f32);
    register_kernel(&k_sobel_thresh_win_f32<2, true>);
    register_kernel(&k_sobel_thresh_win_f32<2, false>);
    register_kernel(&k_sobel_thresh_win_f32<4, true>);
    register_kernel(&k_sobel_thresh_win_f32<4, false>);
    register_kernel(&k_sobel_final);
    register_kernel(&k_saxpy_tanh_sum_f32);
    register_kernel(&k_vec_final);
    register_kernel(&k_vec_batch_tiles<128>);
    register_kernel(&k_vec_batch_tiles<256>);
    register_kernel(&k_vec_batch_tiles<512>);
    register_kernel(&k_vec_batch_tiles<1024>);
    register_kernel(&k_vec_batch_final);
    register_kernel(&k_scan_reduce_i32);
    register_kernel(&k_scan_spine_i64);
    register_kernel(&k_scan_down_i32_i64);
  }
} g_register;
}  // namespace
}  // namespace setrt
