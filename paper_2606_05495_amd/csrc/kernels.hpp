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
  uint32_t* counter;
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
  uint32_t* counter;
  uint32_t* out_count; // output payload
  float* out_sum;
  SlotConst sc;
};
struct VecArgs {
  const float* x;      // pool base
  const float* y;
  float* partials;     // [grid]
  uint32_t* counter;
  float* out_sum;
  SlotConst sc;
  JobScalars js;       // n, a, x_off, y_off
};
struct ScanArgs {
  const int32_t* in;
  void* out;           // int64[n], or uint32[n] low words
  uint32_t* tile_status;  // [ntiles] (epoch << 2) | state
  int64_t* tile_agg;      // [ntiles] tile sums
  int64_t* tile_inc;      // [ntiles] inclusive prefixes
  uint32_t* tile_counter;
  uint32_t* done_counter;
  uint32_t* err;          // set when a look-back exceeded its spin bound
  int low32;
  SlotConst sc;
  JobScalars js;       // n, seq (epoch)
};

__global__ void k_box3_u8_u16(BoxArgs a);
__global__ void k_div9_u16_u8(Div9Args a);
__global__ void k_hist256_u8(HistArgs a);
__global__ void k_gauss5_f32(GaussArgs a);
__global__ void k_sobel_thresh_f32(SobelArgs a);
__global__ void k_saxpy_tanh_sum_f32(VecArgs a);
__global__ void k_scan_i32_i64(ScanArgs a);

}  // namespace setrt
