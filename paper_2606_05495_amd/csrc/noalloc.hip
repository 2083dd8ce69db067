// Vector jobs with no allocation: set_run_vector_jobs_noalloc.
//
// The same bucketed persistent computation as set_run_vector_jobs (per job
// S = sum tanh(a*x + y) over pool windows, split into work items whose size
// is chosen per size bucket floor(log2 n)), for callers that cannot allocate
// device or pinned memory: code under graph capture, tight serving loops.
// Jobs and results are caller-owned device arrays and the call is ordered on
// the caller's stream; the work-item table, the per-item partials and the
// work counter live in one static device array per GPU, whose address is
// looked up once per device.
//
// Three launches on the caller's stream:
//   plan   (one block): validate each job, pick its item size, prefix-sum the
//          item counts into a descriptor table and rewind the work counter;
//   items  (persistent grid): the batch pipeline's (job, item) kernel;
//   totals (one thread per job): each job's item partials in item order.
// A job's result depends only on (n, its item size), as on the batch path,
// so both calls give bit-identical sums for the same jobs and tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <string>

#include "kernels.hpp"

namespace setrt {
namespace {

constexpr uint32_t kNaMaxJobs = SET_NOALLOC_MAX_JOBS;
constexpr uint32_t kNaMaxItems = SET_NOALLOC_MAX_ITEMS;
constexpr int kNaPlanThreads = 1024;
constexpr int kNaMaxDevices = 64;

// Byte offsets inside the static array (each 256-byte aligned).
constexpr uint64_t kNaHdrOff = 0;        // DevSlotHdr the item kernel stamps
constexpr uint64_t kNaWorkOff = 64;      // uint32 work-item counter
constexpr uint64_t kNaTabOff = 256;      // VecBatchHdr + VecBatchDesc[kNaMaxJobs]
constexpr uint64_t kNaTabBytes = (sizeof(VecBatchHdr) + sizeof(VecBatchDesc) * (uint64_t)kNaMaxJobs + 255) / 256 * 256;
constexpr uint64_t kNaPartOff = kNaTabOff + kNaTabBytes;  // float[kNaMaxItems]
constexpr uint64_t kNaBytes = kNaPartOff + 4ull * kNaMaxItems;

}  // namespace
}  // namespace setrt

// The static work area.  In host code this name is only a stand-in for the
// symbol: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[setrt::kNaBytes];

namespace setrt {
namespace {

struct NaPlanArgs {
  const set_vec_job* jobs;
  uint32_t count;
  uint32_t pad;
  uint64_t max_n;
  uint64_t pool_len;
  uint8_t* tab;
  uint32_t* work;
  uint32_t item_elems[64];  // elements per work item, per size bucket
};

struct NaTotalsArgs {
  const uint8_t* tab;
  const float* partials;
  float* results;
};

// Block-wide exclusive prefix of one value per thread (kNaPlanThreads
// threads); *total receives the block's sum.
__device__ inline uint32_t block_excl_u32(uint32_t v, uint32_t* s_wave, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(incl, off, 64);
    if (lane >= off) incl += u;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int k = 0; k < kNaPlanThreads / 64; ++k) {
    const uint32_t t = s_wave[k];
    if (k < wave) before += t;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

__global__ __launch_bounds__(kNaPlanThreads) void k_vec_noalloc_plan(NaPlanArgs a) {
  __shared__ uint32_t s_wave[kNaPlanThreads / 64];
  VecBatchDesc* D = reinterpret_cast<VecBatchDesc*>(a.tab + sizeof(VecBatchHdr));
  uint32_t carry = 0;
  for (uint32_t base = 0; base < a.count; base += kNaPlanThreads) {
    const uint32_t j = base + threadIdx.x;
    VecBatchDesc d{};
    if (j < a.count) {
      const set_vec_job v = a.jobs[j];
      const bool ok = v.n >= 1 && v.n <= a.max_n && v.x_off <= a.pool_len && v.n <= a.pool_len - v.x_off &&
                      v.y_off <= a.pool_len && v.n <= a.pool_len - v.y_off;
      if (ok) {
        const uint32_t te = a.item_elems[63 - __builtin_clzll(v.n)];
        d.x_off = v.x_off;
        d.y_off = v.y_off;
        d.n = (uint32_t)v.n;
        d.a = v.a;
        d.ntiles = (uint32_t)((v.n + te - 1) / te);
        d.tile_elems = te;
      }
    }
    uint32_t chunk_total;
    const uint32_t excl = block_excl_u32(d.ntiles, s_wave, &chunk_total);
    d.tile_start = carry + excl;
    if (j < a.count) D[j] = d;
    carry += chunk_total;
  }
  if (threadIdx.x == 0) {
    VecBatchHdr* H = reinterpret_cast<VecBatchHdr*>(a.tab);
    H->count = a.count;
    H->total_tiles = carry;
    *a.work = 0u;
  }
}

// Job j = thread j: NaN for a job the plan rejected (n == 0 in its
// descriptor), else its item partials in item order.
__global__ __launch_bounds__(kBlock) void k_vec_noalloc_totals(NaTotalsArgs a) {
  const VecBatchHdr* H = reinterpret_cast<const VecBatchHdr*>(a.tab);
  const VecBatchDesc* D = reinterpret_cast<const VecBatchDesc*>(a.tab + sizeof(VecBatchHdr));
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= H->count) return;
  const VecBatchDesc d = D[j];
  a.results[j] = d.n == 0 ? __builtin_nanf("") : vec_items_total(a.partials, d.tile_start, d.ntiles);
}

std::mutex g_na_mu;
std::atomic<unsigned char*> g_na_ptr[kNaMaxDevices];

int na_fail(int code, const std::string& msg) {
  set_thread_error(msg);
  return code;
}

// Device address of `scratch` on the current device `dev`, looked up on the
// first call there.
int na_scratch(int dev, unsigned char** out) {
  unsigned char* p = g_na_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> g(g_na_mu);
    p = g_na_ptr[dev].load(std::memory_order_relaxed);
    if (!p) {
      void* q = nullptr;
      const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !q)
        return na_fail(SET_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
      p = static_cast<unsigned char*>(q);
      g_na_ptr[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return SET_OK;
}

int run_noalloc(int device, hipStream_t stream, const float* x, const float* y, uint64_t pool_len, uint64_t max_n,
                const set_vec_job* jobs, uint64_t count, float* results, const set_vec_tuning* tuning, uint32_t grid) {
  set_thread_error("");
  if (!x || !y || (count && (!jobs || !results))) return na_fail(SET_EINVAL, "null pool, jobs or results pointer");
  if (device < 0 || device >= kNaMaxDevices) return na_fail(SET_EINVAL, "device ordinal out of range");
  if (max_n < 1 || max_n > (1ull << 31)) return na_fail(SET_EINVAL, "max_n outside [1, 2^31]");
  if (count > kNaMaxJobs)
    return na_fail(SET_EINVAL, "count " + std::to_string(count) + " above the maximum of " +
                                   std::to_string(kNaMaxJobs) + " jobs per call");
  if (grid > 65535) return na_fail(SET_EINVAL, "grid above 65535");
  NaPlanArgs pa{};
  // Item size per bucket and the most items any job of length <= max_n needs.
  const int top = 63 - __builtin_clzll(max_n);
  uint64_t worst = 0;
  for (int b = 0; b < 64; ++b) {
    const uint32_t te = (tuning && tuning->tile_elems[b]) ? tuning->tile_elems[b] : vec_default_tile(b);
    if (b <= top) {
      if (te == 0 || te % 1024 != 0) return na_fail(SET_EINVAL, "tile_elems must be a positive multiple of 1024");
      const uint64_t nmax = b == 63 ? max_n : std::min<uint64_t>(max_n, (2ull << b) - 1);
      worst = std::max<uint64_t>(worst, (nmax + te - 1) / te);
    }
    pa.item_elems[b] = te;
  }
  if (count * worst > kNaMaxItems)
    return na_fail(SET_EINVAL, std::to_string(count) + " jobs of length up to max_n may need " +
                                   std::to_string(count * worst) + " work items, above the maximum of " +
                                   std::to_string(kNaMaxItems));
  if (count == 0) return SET_OK;

  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e == hipSuccess && prev != device) e = hipSetDevice(device);
  if (e != hipSuccess) return na_fail(SET_EDEVICE, std::string("hipSetDevice failed: ") + hipGetErrorString(e));
  unsigned char* base = nullptr;
  int rc = na_scratch(device, &base);
  if (rc == SET_OK) {
    uint8_t* tab = base + kNaTabOff;
    uint32_t* work = reinterpret_cast<uint32_t*>(base + kNaWorkOff);
    float* partials = reinterpret_cast<float*>(base + kNaPartOff);
    pa.jobs = jobs;
    pa.count = (uint32_t)count;
    pa.max_n = max_n;
    pa.pool_len = pool_len;
    pa.tab = tab;
    pa.work = work;
    hipLaunchKernelGGL(k_vec_noalloc_plan, dim3(1), dim3(kNaPlanThreads), 0, stream, pa);
    JobScalars js{};
    VecBatchArgs va{tab, x, y, partials, work, reinterpret_cast<DevSlotHdr*>(base + kNaHdrOff), js};
    hipLaunchKernelGGL(k_vec_batch_tiles<kBlock>, dim3(grid ? grid : (unsigned)kVecBatchGrid), dim3(kBlock), 0, stream, va);
    NaTotalsArgs ta{tab, partials, results};
    hipLaunchKernelGGL(k_vec_noalloc_totals, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream,
                       ta);
    e = hipGetLastError();
    if (e != hipSuccess) rc = na_fail(SET_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  }
  if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
  return rc;
}

}  // namespace
}  // namespace setrt

extern "C" int set_run_vector_jobs_noalloc(int device, void* stream, const float* dev_x_pool, const float* dev_y_pool,
                                           uint64_t pool_len, uint64_t max_n, const set_vec_job* dev_jobs,
                                           uint64_t count, float* dev_results, const set_vec_tuning* tuning,
                                           uint32_t grid) {
  return setrt::run_noalloc(device, static_cast<hipStream_t>(stream), dev_x_pool, dev_y_pool, pool_len, max_n,
                            dev_jobs, count, dev_results, tuning, grid);
}
