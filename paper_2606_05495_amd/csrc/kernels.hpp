// Stage kernels of the job chains and their argument blocks.  Each kernel
// takes one argument struct by value, so a graph kernel node's per-job
// placeholder (Section 4.1) is a single struct that the binder rewrites.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "tiles.hpp"

namespace setrt {

// Per-slot constants the last stage of every chain needs to publish the
// output header (fixed when the slot is laid out; never rebound).
struct SlotConst {
  DevSlotHdr* hdr;
  const uint64_t* tail;
  set_out_header* outh;
  uint64_t canary_head;
  uint64_t canary_tail;
};

// ---- argument blocks
struct BoxArgs {
  const uint8_t* in;
  uint16_t* S;
  int h, w;
  DevSlotHdr* hdr;
  JobScalars js;
};
struct Div9Args {
  const uint16_t* S;
  uint8_t* Q;
  int64_t npix;
};
struct HistArgs {
  const uint8_t* Q;
  int64_t npix;
  uint32_t* partials;  // [grid][256]
};
struct HistFinalArgs {
  const uint32_t* partials;
  unsigned nblocks;
  uint32_t* H;         // output payload
  SlotConst sc;
};
struct GaussArgs {
  const float* in;
  float* out;
  int h, w;
  float g0, g1, g2;    // taps (g[-2]=g[2]=g0, g[-1]=g[1]=g1, centre g2)
  DevSlotHdr* hdr;
  JobScalars js;
};
struct SobelArgs {
  const float* blur;
  uint8_t* mask;
  int h, w;
  float thr;
  uint32_t* pcount;    // [grid]
  float* psum;         // [grid]
};
struct SobelFinalArgs {
  const uint32_t* pcount;
  const float* psum;
  unsigned nparts;     // partial pairs to combine
  uint32_t* out_count; // output payload
  float* out_sum;
  SlotConst sc;
};
struct VecArgs {
  const float* x;      // pool base
  const float* y;
  float* partials;     // [grid]
  DevSlotHdr* hdr;
  JobScalars js;       // n, a, x_off, y_off
};
struct VecFinalArgs {
  const float* partials;  // [vec_blocks(n)], n read from the slot header
  float* out_sum;
  SlotConst sc;
};
struct VecBatchArgs {
  const uint8_t* tab;  // descriptor table in the slot (VecBatchHdr + VecBatchDesc[count])
  const float* x;
  const float* y;
  float* partials;     // [total_tiles]
  uint32_t* work;      // work-item counter (zero between batches)
  DevSlotHdr* hdr;
  JobScalars js;
};
struct VecBatchFinalArgs {
  const uint8_t* tab;
  const float* partials;
  uint32_t* work;
  float* results;      // output payload, one float per job
  SlotConst sc;
};
// Scan as reduce -> spine -> downsweep; all three are launched with the grid
// of the template's largest n, so a job of any length needs no grid update.
// The reduce and the downsweep take the job's n in their argument blocks; the
// one-block spine reads it from the slot header.
struct ScanReduceArgs {
  const int32_t* in;
  int64_t* tile_sum;   // [tiles]
  unsigned max_tiles;
  DevSlotHdr* hdr;
  JobScalars js;
};
struct ScanSpineArgs {
  const int64_t* tile_sum;
  int64_t* tile_excl;  // [tiles] exclusive prefix of tile sums
  SlotConst sc;
  uint64_t n;          // the job's length, rebound per job like the downsweep's
};
// The downsweep carries the job's n in its own argument block (rebound with
// the first kernel's), so its data loads need no dependent load of the slot
// header first: one memory round trip instead of two.
struct ScanDownArgs {
  const int32_t* in;
  const int64_t* tile_excl;
  void* out;           // int64[n], or uint32[n] low words
  int low32;
  uint64_t n;          // the job's length
};

// Host<->device copy as a kernel: a small grid of 16-byte loads/stores that
// keeps PCIe busy without occupying the whole device.
struct CopyArgs {
  const void* src;
  void* dst;
  uint64_t bytes;
};
__global__ void k_copy_in(CopyArgs a);   // host-to-device
// Bandwidth reference: word i of `nvec` 16-byte words copied by thread i.
struct RefCopyArgs {
  const void* src;
  void* dst;
  uint64_t nvec;
};
__global__ void k_ref_copy(RefCopyArgs a);
__global__ void k_copy_out(CopyArgs a);  // device-to-host

// Completion word: one thread stores the job's binding sequence number (from
// the slot header) into a pinned host word with a system-scope release.
struct DoneFlagArgs {
  const DevSlotHdr* hdr;
  uint64_t* word;
};
__global__ void k_done_flag(DoneFlagArgs a);

// Memory-safety stress (template options).  k_poison runs after a job's
// output copy and fills the slot's buffers (everything between the header
// and the tail canary) with 0xFF bytes, so a job that read anything a
// previous job left in its slot would read NaN / all-ones values; the one
// word the slot carries from job to job on purpose (the work counter of
// batched vector templates, rewound to zero by the job's last stage) is
// written as zero.  k_stress_delay runs before the first stage and sleeps
// until the device's constant-rate clock has advanced by `ticks`, stretching
// the window in which a slot released too early would be overwritten.
struct PoisonArgs {
  void* p;              // 16-byte aligned start of the poisoned range
  uint64_t nvec;        // 16-byte words in the range
  uint64_t zero_word;   // index (uint32 units from p) of the word written as 0, or ~0 for none
};
__global__ void k_poison(PoisonArgs a);
struct DelayArgs {
  uint64_t ticks;       // constant-clock ticks to wait
  uint64_t max_sleeps;  // bound on the sleep loop, so the wait ends whatever the clock reads
};
__global__ void k_stress_delay(DelayArgs a);

// Bracket kernels of a job whose middle stages are library code captured
// into the job graph: the first writes the job's scalars into the slot
// header, the last checks the canaries and publishes the output header.
struct JobBeginArgs {
  DevSlotHdr* hdr;
  JobScalars js;
};
struct JobEndArgs {
  SlotConst sc;
};
__global__ void k_job_begin(JobBeginArgs a);
__global__ void k_job_end(JobEndArgs a);

// The library stage of a library-call template: rocPRIM's device-wide
// inclusive scan of n int32 values into int64 sums, widening on load, on
// stream st (lib_scan.hip).  With ws == nullptr only ws_bytes is computed.
hipError_t lib_scan(void* ws, size_t& ws_bytes, const int32_t* in, int64_t* out, size_t n, hipStream_t st);

// One explicit step of the thermal grid: tout = step(tin, p).  The first
// step of a job (first != 0) also writes the job's scalars into the slot
// header.
struct HotspotArgs {
  const float* tin;
  const float* p;
  float* tout;
  int h, w;
  int first;
  DevSlotHdr* hdr;
  JobScalars js;
};
template <bool FULL>
__global__ void k_hotspot_win_f32(HotspotArgs a);
template <int R>
__global__ void k_hotspot_band_f32(HotspotArgs a);
__global__ void k_hotspot_f32(HotspotArgs a);

__global__ void k_box3_u8_u16(BoxArgs a);
__global__ void k_div9_u16_u8(Div9Args a);
__global__ void k_hist256_u8(HistArgs a);
__global__ void k_hist256_final(HistFinalArgs a);
__global__ void k_gauss5_f32(GaussArgs a);
template <int R, bool FULL>
__global__ void k_gauss5_win_f32(GaussArgs a);
template <int R>
__global__ void k_gauss5_band_f32(GaussArgs a);
__global__ void k_sobel_thresh_f32(SobelArgs a);
template <int R, bool FULL>
__global__ void k_sobel_thresh_win_f32(SobelArgs a);
__global__ void k_sobel_final(SobelFinalArgs a);
__global__ void k_saxpy_tanh_sum_f32(VecArgs a);
__global__ void k_vec_final(VecFinalArgs a);
// Sum of one vector job's work-item partials in item order: the fixed order
// that makes a job's result depend only on its length and item size.
__device__ inline float vec_items_total(const float* partials, uint32_t first, uint32_t count) {
  float s = 0.f;
  for (uint32_t k = 0; k < count; ++k) s += partials[first + k];
  return s;
}

// BLOCK threads per block: 128, 256, 512 or 1024 (the template's block).
template <int BLOCK>
__global__ void k_vec_batch_tiles(VecBatchArgs a);
__global__ void k_vec_batch_final(VecBatchFinalArgs a);
__global__ void k_scan_reduce_i32(ScanReduceArgs a);
__global__ void k_scan_spine_i64(ScanSpineArgs a);
__global__ void k_scan_down_i32_i64(ScanDownArgs a);

}  // namespace setrt
