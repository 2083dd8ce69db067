// Stage kernels for CDNA4 (gfx950), wave64.  No MFMA: nothing here is a dense
// contraction.  Image stages stage their tile plus halo in LDS; reductions use
// wave shuffles and LDS in a fixed order, so every result depends only on the
// job's input and size (bit-identical whatever stream, slot or neighbour ran
// beside it); the histogram uses LDS atomics on per-wave private bins.
//
// Cross-block results are combined by a separate single-block kernel node
// that runs after the producing kernel has finished (the kernel boundary is
// the only synchronisation: no per-block device-scope fences, which on this
// multi-XCD part write back the issuing XCD's L2 and cost tens of
// microseconds when a thousand blocks issue them).  That last kernel combines
// the per-block partials in block order, checks the slot's canaries and
// publishes the output header.
#include <type_traits>

#include "kernels.hpp"

namespace setrt {

// ------------------------------------------------------------------ helpers
__device__ inline void write_slot_hdr(DevSlotHdr* hdr, const JobScalars& js) {
  hdr->job_id = js.job_id;
  hdr->seq = js.seq;
  hdr->user_tag = js.user_tag;
  hdr->worker = js.worker;
  hdr->slot = js.slot;
  hdr->n = js.n;
}

// One thread; the caller has acquired everything the job wrote.  The two
// canary tests are combined without short-circuit, so every load of the
// header and the tail goes out at once: one memory round trip.
__device__ inline void publish_out(const SlotConst& sc, bool extra_ok) {
  const DevSlotHdr* h = sc.hdr;
  set_out_header* o = sc.outh;
  const bool canaries = (h->canary_head == sc.canary_head) & (*sc.tail == sc.canary_tail);
  o->job_id = h->job_id;
  o->seq = h->seq;
  o->worker = h->worker;
  o->slot = h->slot;
  o->user_tag = h->user_tag;
  o->canary_ok = canaries ? 1u : 0u;
  o->reserved[0] = 0;
  o->reserved[1] = 0;
  o->reserved[2] = 0;
  o->magic = extra_ok ? SET_OUT_MAGIC : 0xBAD0BAD0u;
}

__device__ inline float wave_sum_f32(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sums in a fixed order: lane 0 of each wave, then waves 0..3 pairwise.
// Every thread returns the same value.
__device__ inline float block_sum_f32(float v, float* s4) {
  v = wave_sum_f32(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s4[wave] = v;
  __syncthreads();
  return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}
__device__ inline uint32_t block_sum_u32(uint32_t v, uint32_t* s4) {
  v = wave_sum_u32(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s4[wave] = v;
  __syncthreads();
  return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Stage outputs (the blurred image, the mask, a heat step's grid, the scan's
// sums) are stored with the nontemporal hint.  On cold buffers this takes the
// Gaussian from 4.12 to 3.60 us at 1024x1024 and from 9.19 to 8.62 us at
// 2048x2048, Sobel from 6.36 to 6.01 us and the heat step from 10.69 to
// 10.15 us at 2048x2048; the next stage, which reads them, did not slow
// (thermal jobs of 16 steps ran at the same rate either way).
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef long long v2i64_t __attribute__((ext_vector_type(2)));
typedef unsigned v4u_t __attribute__((ext_vector_type(4)));
__device__ inline void store_nt(float* p, float x, float y, float z, float w) {
  __builtin_nontemporal_store(v4f_t{x, y, z, w}, reinterpret_cast<v4f_t*>(p));
}
__device__ inline void store_nt(int64_t* p, int64_t x, int64_t y) {
  __builtin_nontemporal_store(v2i64_t{x, y}, reinterpret_cast<v2i64_t*>(p));
}
__device__ inline void store_nt(uint32_t* p, uint32_t x, uint32_t y, uint32_t z, uint32_t w) {
  __builtin_nontemporal_store(v4u_t{x, y, z, w}, reinterpret_cast<v4u_t*>(p));
}
__device__ inline void store_nt(uint32_t* p, uint32_t x) { __builtin_nontemporal_store(x, p); }
// Global-memory (address space 1) views of an integer address.  A row base
// held in scalar registers as an integer, plus a lane's 32-bit byte offset,
// then loads and stores as global_load/store with a scalar base, where the
// compiler would otherwise form one 64-bit vector address per row.
typedef v4f_t __attribute__((address_space(1))) GlobalV4f;
typedef const float __attribute__((address_space(1))) GlobalF32;
__device__ inline v4f_t make_v4f(float x, float y, float z, float w) { return v4f_t{x, y, z, w}; }

// The hardware square root (v_sqrt_f32, within 1 ulp for normal inputs)
// instead of the correctly rounded library sequence, which costs about 15
// instructions per call; the Sobel magnitudes here are normal numbers and
// their parity bound is 1e-5 relative.
__device__ inline float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }

// Fill an LDS tile of N elements (row-major, LW per row, stored with pitch
// P) from global memory: every thread issues all of its loads before its
// first LDS write, so one memory latency covers the whole tile.  get(r, c)
// returns the element for tile row r, column c.
template <typename T, int LW, int LH, int P, class Get>
__device__ inline void stage_tile(T (*tile)[P], Get get) {
  constexpr int N = LW * LH;
  constexpr int PER = (N + kBlock - 1) / kBlock;
  T vals[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + k * kBlock;
    const int r = i / LW, c = i - r * LW;
    vals[k] = (i < N) ? get(r, c) : T(0);
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + k * kBlock;
    const int r = i / LW, c = i - r * LW;
    if (i < N) tile[r][c] = vals[k];
  }
}

// ------------------------------------------------------------------ copy kernels (H2D pull / D2H push)
// Grid-stride over 16-byte words with four independent loads in flight per
// thread, then a byte tail.  Source and destination are 16-byte aligned (slot
// buffers are 256-aligned; host buffers are checked by the binder).  The two
// directions are separate kernels only so that a kernel trace tells them
// apart (input-copy idle time, batch boundaries).
__device__ __forceinline__ void copy_bytes(const CopyArgs& a) {
  const uint64_t nvec = a.bytes >> 4;
  const uint4* __restrict__ src = reinterpret_cast<const uint4*>(a.src);
  uint4* __restrict__ dst = reinterpret_cast<uint4*>(a.dst);
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  for (; i + 3 * stride < nvec; i += 4 * stride) {
    const uint4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
    dst[i] = v0;
    dst[i + stride] = v1;
    dst[i + 2 * stride] = v2;
    dst[i + 3 * stride] = v3;
  }
  for (; i < nvec; i += stride) dst[i] = src[i];
  const uint64_t tail = nvec << 4;
  const uint64_t t = tail + (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < a.bytes) reinterpret_cast<uint8_t*>(a.dst)[t] = reinterpret_cast<const uint8_t*>(a.src)[t];
}
__global__ __launch_bounds__(kBlock) void k_copy_in(CopyArgs a) { copy_bytes(a); }
__global__ __launch_bounds__(kBlock) void k_ref_copy(RefCopyArgs a) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < a.nvec) static_cast<uint4*>(a.dst)[i] = static_cast<const uint4*>(a.src)[i];
}
__global__ __launch_bounds__(kBlock) void k_copy_out(CopyArgs a) { copy_bytes(a); }

// ------------------------------------------------------------------ completion word
// Runs after the job's device-to-host copy node; the kernel boundary orders
// the copy's host writes before this store.
__global__ __launch_bounds__(64) void k_done_flag(DoneFlagArgs a) {
  if (threadIdx.x == 0) __hip_atomic_store(a.word, a.hdr->seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ------------------------------------------------------------------ memory-safety stress
__global__ __launch_bounds__(kBlock) void k_poison(PoisonArgs a) {
  const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u);
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint64_t zv = a.zero_word >> 2;  // the 16-byte word that holds the zero word, if any
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < a.nvec; i += stride) {
    uint4 v = ones;
    if (i == zv) {
      const unsigned c = (unsigned)(a.zero_word & 3);
      v.x = c == 0 ? 0u : v.x;
      v.y = c == 1 ? 0u : v.y;
      v.z = c == 2 ? 0u : v.z;
      v.w = c == 3 ? 0u : v.w;
    }
    reinterpret_cast<uint4*>(a.p)[i] = v;
  }
}

// One wave; s_sleep 8 is 512 clocks, so the loop ends within max_sleeps
// iterations even if the clock does not advance.
__global__ __launch_bounds__(64) void k_stress_delay(DelayArgs a) {
  if (threadIdx.x != 0) return;
  const uint64_t t0 = (uint64_t)wall_clock64();
  for (uint64_t k = 0; k < a.max_sleeps && (uint64_t)wall_clock64() - t0 < a.ticks; ++k)
    __builtin_amdgcn_s_sleep(8);
}

// ------------------------------------------------------------------ bracket kernels of library-call jobs
__global__ __launch_bounds__(kBlock) void k_job_begin(JobBeginArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, a.js);
}
__global__ __launch_bounds__(kBlock) void k_job_end(JobEndArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) publish_out(a.sc, true);
}

// ------------------------------------------------------------------ 3x3 box sum (zero padded), uint8 -> uint16
// Output tile kBoxTW x kBoxTH, input tile + 1-pixel halo staged in LDS.
__global__ __launch_bounds__(kBlock) void k_box3_u8_u16(BoxArgs a) {
  constexpr int LW = kBoxTW + 2, LH = kBoxTH + 2;
  __shared__ uint8_t tile[LH][LW + 2];
  const int x0 = blockIdx.x * kBoxTW, y0 = blockIdx.y * kBoxTH;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, a.js);
  stage_tile<uint8_t, LW, LH, LW + 2>(tile, [&](int r, int c) {
    const int gy = y0 + r - 1, gx = x0 + c - 1;
    return (gy >= 0 && gy < a.h && gx >= 0 && gx < a.w) ? a.in[(size_t)gy * a.w + gx] : (uint8_t)0;
  });
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int y = y0 + ty;
  if (y >= a.h) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int lx = tx * 4 + k, x = x0 + lx;
    if (x < a.w) {
      unsigned s = 0;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) s += tile[ty + dy][lx + dx];
      a.S[(size_t)y * a.w + x] = (uint16_t)s;
    }
  }
}

// ------------------------------------------------------------------ floor(s / 9), uint16 -> uint8
__global__ __launch_bounds__(kBlock) void k_div9_u16_u8(Div9Args a) {
  const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kDivPerThread;
  if (i0 + kDivPerThread <= a.npix) {
    const uint4 v = *reinterpret_cast<const uint4*>(a.S + i0);  // 8 x uint16, 16-byte aligned
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    uint32_t o[2] = {0u, 0u};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t lo = (w[k] & 0xFFFFu) / 9u, hi = (w[k] >> 16) / 9u;
      o[k >> 1] |= (lo | (hi << 8)) << (16 * (k & 1));
    }
    *reinterpret_cast<uint2*>(a.Q + i0) = make_uint2(o[0], o[1]);
  } else {
    for (int64_t i = i0; i < a.npix; ++i) a.Q[i] = (uint8_t)(a.S[i] / 9u);
  }
}

// ------------------------------------------------------------------ 256-bin histogram of uint8
// Per-wave private LDS bins (4 x 256) take the LDS atomics; the block's sum of
// them goes to partials[block].
__global__ __launch_bounds__(kBlock) void k_hist256_u8(HistArgs a) {
  __shared__ uint32_t wh[4][256];
  const int tid = threadIdx.x, wave = tid >> 6;
  for (int i = tid; i < 4 * 256; i += kBlock) (&wh[0][0])[i] = 0u;
  __syncthreads();
  const int64_t base = ((int64_t)blockIdx.x * kBlock + tid) * kHistPerThread;
  if (base + kHistPerThread <= a.npix) {
    const uint4 v = *reinterpret_cast<const uint4*>(a.Q + base);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int b = 0; b < 4; ++b) atomicAdd(&wh[wave][(w[k] >> (8 * b)) & 255u], 1u);
  } else {
    for (int64_t i = base; i < a.npix; ++i) atomicAdd(&wh[wave][a.Q[i]], 1u);
  }
  __syncthreads();
  a.partials[(size_t)blockIdx.x * 256 + tid] = wh[0][tid] + wh[1][tid] + wh[2][tid] + wh[3][tid];
}

// One block: bin tid = sum of the blocks' partial counts (integer, exact in
// any order).  The loads go out 16 blocks at a time with no branch between
// them (past the last block the index is clamped and the value dropped), so
// one memory latency covers 16 blocks instead of one.
__global__ __launch_bounds__(kBlock) void k_hist256_final(HistFinalArgs a) {
  const int tid = threadIdx.x;
  const unsigned nb = a.nblocks;
  uint32_t s = 0;
  for (unsigned b0 = 0; b0 < nb; b0 += 16) {
    uint32_t v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const unsigned b = b0 + k < nb ? b0 + k : nb - 1;
      v[k] = a.partials[(size_t)b * 256 + tid];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) s += b0 + k < nb ? v[k] : 0u;
  }
  a.H[tid] = s;
  if (tid == 0) publish_out(a.sc, true);
}

// ------------------------------------------------------------------ separable 5-tap Gaussian, replicated borders
// Input tile (kGaussTH+4) x (kGaussTW+4) in LDS, horizontal pass into a
// second LDS tile (kGaussTH+4) x kGaussTW, vertical pass to global.
__global__ __launch_bounds__(kBlock) void k_gauss5_f32(GaussArgs a) {
  constexpr int IW = kGaussTW + 4, IH = kGaussTH + 4;
  __shared__ float tin[IH][IW + 1];
  __shared__ float tmid[IH][kGaussTW + 1];
  const int x0 = blockIdx.x * kGaussTW, y0 = blockIdx.y * kGaussTH;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, a.js);
  const int wm = a.w - 1, hm = a.h - 1;
  stage_tile<float, IW, IH, IW + 1>(tin, [&](int r, int c) {
    return a.in[(size_t)clampi(y0 + r - 2, 0, hm) * a.w + clampi(x0 + c - 2, 0, wm)];
  });
  __syncthreads();
  const float g0 = a.g0, g1 = a.g1, g2 = a.g2;
  for (int i = threadIdx.x; i < IH * kGaussTW; i += kBlock) {
    const int r = i / kGaussTW, c = i - r * kGaussTW;
    float acc = g0 * tin[r][c];
    acc = fmaf(g1, tin[r][c + 1], acc);
    acc = fmaf(g2, tin[r][c + 2], acc);
    acc = fmaf(g1, tin[r][c + 3], acc);
    acc = fmaf(g0, tin[r][c + 4], acc);
    tmid[r][c] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kGaussTH * kGaussTW; i += kBlock) {
    const int r = i / kGaussTW, c = i - r * kGaussTW;
    const int y = y0 + r, x = x0 + c;
    if (y < a.h && x < a.w) {
      float acc = g0 * tmid[r][c];
      acc = fmaf(g1, tmid[r + 1][c], acc);
      acc = fmaf(g2, tmid[r + 2][c], acc);
      acc = fmaf(g1, tmid[r + 3][c], acc);
      acc = fmaf(g0, tmid[r + 4][c], acc);
      a.out[(size_t)y * a.w + x] = acc;
    }
  }
}

// ------------------------------------------------------------------ Sobel magnitude + threshold + count/sum
// gx = (right column) - (left column) with weights 1,2,1; gy = (row below) -
// (row above); mag = sqrt(gx^2 + gy^2); mask = mag > thr.  Each block writes
// its count and its magnitude sum (fixed-order block reduction).
__global__ __launch_bounds__(kBlock) void k_sobel_thresh_f32(SobelArgs a) {
  constexpr int IW = kSobelTW + 2, IH = kSobelTH + 2;
  __shared__ float t[IH][IW + 1];
  __shared__ float s4f[4];
  __shared__ uint32_t s4u[4];
  const int x0 = blockIdx.x * kSobelTW, y0 = blockIdx.y * kSobelTH;
  const int wm = a.w - 1, hm = a.h - 1;
  stage_tile<float, IW, IH, IW + 1>(t, [&](int r, int c) {
    return a.blur[(size_t)clampi(y0 + r - 1, 0, hm) * a.w + clampi(x0 + c - 1, 0, wm)];
  });
  __syncthreads();
  float sum = 0.f;
  uint32_t cnt = 0;
  for (int i = threadIdx.x; i < kSobelTH * kSobelTW; i += kBlock) {
    const int r = i / kSobelTW, c = i - r * kSobelTW;
    const int y = y0 + r, x = x0 + c;
    if (y < a.h && x < a.w) {
      const float p00 = t[r][c], p01 = t[r][c + 1], p02 = t[r][c + 2];
      const float p10 = t[r + 1][c], p12 = t[r + 1][c + 2];
      const float p20 = t[r + 2][c], p21 = t[r + 2][c + 1], p22 = t[r + 2][c + 2];
      const float gx = (p02 + 2.f * p12 + p22) - (p00 + 2.f * p10 + p20);
      const float gy = (p20 + 2.f * p21 + p22) - (p00 + 2.f * p01 + p02);
      const float mag = sqrt_hw(gx * gx + gy * gy);
      const uint32_t on = mag > a.thr ? 1u : 0u;
      a.mask[(size_t)y * a.w + x] = (uint8_t)on;
      cnt += on;
      sum += mag;
    }
  }
  const unsigned b = blockIdx.y * gridDim.x + blockIdx.x;
  const float bs = block_sum_f32(sum, s4f);
  const uint32_t bc = block_sum_u32(cnt, s4u);
  if (threadIdx.x == 0) {
    a.psum[b] = bs;
    a.pcount[b] = bc;
  }
}

// ------------------------------------------------------------------ register-window image kernels
// Path for float images whose width is a multiple of 4.  A lane owns 4
// adjacent columns (one 16-byte load or store per row), a wave 256 columns,
// and slides down R output rows with the window of input rows in
// registers: every input row of the wave is loaded before the first result
// is formed, so each wave has all its loads in flight at once.  Neighbouring
// columns come from the adjacent lanes by whole-wave lane shifts; lanes 0 and
// 63 take the columns beyond the wave from extra (clamped) loads.  A block is
// 4 waves stacked vertically.
//
// Blocks are dealt to the 8 XCDs round-robin in launch order.  xcd_tile
// renumbers them so each XCD owns a contiguous run of tiles in row-major
// order: vertically adjacent tiles, which read each other's halo rows, then
// share one L2.
__device__ inline void xcd_tile(unsigned& bx, unsigned& by) {
  const unsigned gx = gridDim.x, n = gx * gridDim.y;
  const unsigned L = blockIdx.y * gx + blockIdx.x;
  const unsigned q = n >> 3, rem = n & 7u, x = L & 7u, k = L >> 3;
  const unsigned t = x * q + (x < rem ? x : rem) + k;  // XCD x owns tiles [x*q + min(x, rem), ...)
  by = t / gx;
  bx = t - by * gx;
}

// Whole-wave shifts by one lane (DPP wave_shr:1 / wave_shl:1, a VALU move
// instead of an LDS permute).  from_left gives lane i the value of lane i-1,
// from_right the value of lane i+1.  With bound_ctrl off, the lane whose
// source lies outside the wave (lane 0 for from_left, lane 63 for
// from_right) keeps the old value, which is its own `edge`: the tile's halo
// column arrives without a per-lane select.
__device__ inline float from_left(float v, float edge) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ inline float from_right(float v, float edge) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130, 0xf, 0xf, false));
}

// Sum over the wave in six DPP steps: two quad permutes, the half-row and row
// mirrors (each lane then holds its 16-lane row's sum), then row_bcast:15 into
// rows 1 and 3 and row_bcast:31 into rows 2 and 3; lane 63 ends with the total,
// which readlane returns to every lane.  Lanes of rows a broadcast leaves out
// add the old value 0.  The order of the additions is fixed.
template <int CTRL, int ROWS = 0xf>
__device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);
}
__device__ inline float wave_total_f32(float v) {
  v += __int_as_float(dpp_i<0xb1>(__float_as_int(v)));        // quad_perm [1,0,3,2]
  v += __int_as_float(dpp_i<0x4e>(__float_as_int(v)));        // quad_perm [2,3,0,1]
  v += __int_as_float(dpp_i<0x141>(__float_as_int(v)));       // row_half_mirror
  v += __int_as_float(dpp_i<0x140>(__float_as_int(v)));       // row_mirror
  v += __int_as_float(dpp_i<0x142, 0xa>(__float_as_int(v)));  // row_bcast:15
  v += __int_as_float(dpp_i<0x143, 0xc>(__float_as_int(v)));  // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ inline uint32_t wave_total_u32(uint32_t v) {
  int x = (int)v;
  x += dpp_i<0xb1>(x);
  x += dpp_i<0x4e>(x);
  x += dpp_i<0x141>(x);
  x += dpp_i<0x140>(x);
  x += dpp_i<0x142, 0xa>(x);
  x += dpp_i<0x143, 0xc>(x);
  return (uint32_t)__builtin_amdgcn_readlane(x, 63);
}

// Register-window geometry of one lane.  The wave index goes through
// readfirstlane, so the wave's rows (and every row address, clamp and bounds
// test derived from them) live in scalar registers; a load or store is then a
// scalar row base plus the lane's 32-bit byte offset.  FULL: the width is a
// multiple of 256, so every lane's 4 columns lie inside the image.  Otherwise
// lanes past the right edge load the last 4 columns and keep only the border
// column (replicated), and store nothing.
template <bool FULL>
struct WinLane {
  int lane, y0;       // y0: first output row of the wave (wave-uniform)
  unsigned x;         // first of the lane's 4 columns
  unsigned xl;        // column the lane loads from
  bool past;          // lane lies beyond the right edge (never when FULL)
  __device__ WinLane(int w, unsigned bx, unsigned by, int rows) {
    lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    y0 = ((int)by * 4 + wave) * rows;
    x = bx * kWinCols + 4u * lane;
    past = FULL ? false : x >= (unsigned)w;
    xl = past ? (unsigned)w - 4u : x;
  }
  __device__ float4 load4(const float* row) const {
    const float4 t = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(row) + xl * 4u);
    return past ? make_float4(t.w, t.w, t.w, t.w) : t;
  }
};
__device__ inline float load1(const float* row, unsigned col) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(row) + col * 4u);
}

// Separable 5-tap Gaussian on the register window, vertical pass first: each
// lane filters its own 4 columns down the R + 4 loaded rows (and lanes 0 and
// 63 the two columns beyond the wave's edge), then the horizontal pass takes
// the neighbouring columns' vertical results by lane shift.  Vertical first
// costs (R + 4)/R fewer lane shifts and FMAs than horizontal first, since the
// horizontal pass then runs on R rows instead of R + 4.
template <int R, bool FULL>
__global__ __launch_bounds__(kBlock) void k_gauss5_win_f32(GaussArgs a) {
  unsigned bx, by;
  xcd_tile(bx, by);
  if (bx == 0 && by == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, a.js);
  const int w = a.w, h = a.h, wm = w - 1, hm = h - 1;
  const WinLane<FULL> L(w, bx, by, R);
  const int xw = (int)bx * kWinCols;
  // lane 0 needs columns xw-2, xw-1; lane 63 needs xw+256, xw+257
  const unsigned hx0 = clampi(L.lane == 0 ? xw - 2 : xw + kWinCols, 0, wm);
  const unsigned hx1 = clampi(L.lane == 0 ? xw - 1 : xw + kWinCols + 1, 0, wm);
  float4 v[R + 4];
  float e0[R + 4], e1[R + 4];
#pragma unroll
  for (int r = 0; r < R + 4; ++r) {
    const float* row = a.in + (size_t)clampi(L.y0 + r - 2, 0, hm) * w;
    v[r] = L.load4(row);
    e0[r] = load1(row, hx0);
    e1[r] = load1(row, hx1);
  }
  const float g0 = a.g0, g1 = a.g1, g2 = a.g2;
  auto vert = [&](float t0, float t1, float t2, float t3, float t4) {
    float acc = g0 * t0;
    acc = fmaf(g1, t1, acc);
    acc = fmaf(g2, t2, acc);
    acc = fmaf(g1, t3, acc);
    return fmaf(g0, t4, acc);
  };
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float c0 = vert(v[r].x, v[r + 1].x, v[r + 2].x, v[r + 3].x, v[r + 4].x);
    const float c1 = vert(v[r].y, v[r + 1].y, v[r + 2].y, v[r + 3].y, v[r + 4].y);
    const float c2 = vert(v[r].z, v[r + 1].z, v[r + 2].z, v[r + 3].z, v[r + 4].z);
    const float c3 = vert(v[r].w, v[r + 1].w, v[r + 2].w, v[r + 3].w, v[r + 4].w);
    const float f0 = vert(e0[r], e0[r + 1], e0[r + 2], e0[r + 3], e0[r + 4]);
    const float f1 = vert(e1[r], e1[r + 1], e1[r + 2], e1[r + 3], e1[r + 4]);
    const float c[8] = {from_left(c2, f0), from_left(c3, f1), c0, c1, c2, c3, from_right(c0, f0), from_right(c1, f1)};
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = vert(c[j], c[j + 1], c[j + 2], c[j + 3], c[j + 4]);
    const int y = L.y0 + r;
    if (y < h && !L.past)
      store_nt(reinterpret_cast<float*>(reinterpret_cast<char*>(a.out + (size_t)y * w) + L.x * 4u), o[0], o[1], o[2],
               o[3]);
  }
}
// Row bands, for widths that are a multiple of kBandCols: a block of
// kBandCols / 256 waves lies side by side across R whole rows (8, or 4 above
// 4096^2 pixels), each wave 256 columns as in the window kernel.  A wave's halo columns are
// its neighbours' outermost columns, whose vertical-pass results the
// neighbours already hold: each wave's lane 0 publishes its first two columns
// and lane 63 its last two in LDS, and after one barrier lanes 0 and 63 read
// the neighbouring waves' pairs.  Only the block's outer edges, where they lie
// inside the image, load their two halo columns (the first wave on the left,
// the last on the right); at the image border the clamped columns are the
// border column itself, whose vertical result the border lane already holds.
// Against the window kernel at 4 rows, which loads both halo pairs in every
// wave, a wave issues R + 4 vector loads instead of 3 (R + 4) and skips two
// columns' vertical passes, and at 8 rows it re-reads 1.5x its rows from L2
// instead of 2x; the barrier makes a wave wait for its block's slowest load,
// which costs more than that saves on images of a million pixels or fewer,
// where each SIMD holds one wave.  The arithmetic is the window kernel's,
// operation for operation.
template <int R>
__global__ __launch_bounds__(kBandCols / 4) void k_gauss5_band_f32(GaussArgs a) {
  constexpr int nw = kBandCols / kWinCols;
  unsigned bx, band;
  xcd_tile(bx, band);  // grid (column blocks, bands)
  if (bx == 0 && band == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, a.js);
  // lo[k + 1][r]: wave k's two first columns; hi[k + 1][r]: its two last.
  // hi[0] holds the pair left of the block, lo[nw + 1] the pair right of it.
  __shared__ float2 lo[nw + 2][R], hi[nw + 2][R];
  const int w = a.w, h = a.h, hm = h - 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int y0 = (int)band * R;
  const unsigned xb = bx * (unsigned)kBandCols;  // first column of the block
  const unsigned x = xb + (unsigned)wave * kWinCols + 4u * (unsigned)lane;
  const uint32_t pitch = (uint32_t)w * 4u;  // row bytes
  const bool left_out = wave == 0 && bx > 0;                    // halo left of the block inside the image
  const bool right_out = wave == nw - 1 && bx + 1 < gridDim.x;  // halo right of the block inside the image
  auto row_base = [&](const float* img, int r) {
    uint64_t row = reinterpret_cast<uint64_t>(img) + (uint64_t)(uint32_t)clampi(y0 + r - 2, 0, hm) * pitch;
    asm("" : "+s"(row));  // keeps the row base scalar: scalar base + 32-bit lane offset per load
    return row;
  };
  float e0[R + 4], e1[R + 4];
  if (left_out || right_out) {  // wave-uniform (same address in every lane), issued before the window rows
    const unsigned hc = (left_out ? xb - 2u : xb + (unsigned)kBandCols) * 4u;
#pragma unroll
    for (int r = 0; r < R + 4; ++r) {
      const uint64_t row = row_base(a.in, r);
      e0[r] = *reinterpret_cast<const GlobalF32*>(row + hc);
      e1[r] = *reinterpret_cast<const GlobalF32*>(row + hc + 4u);
    }
  }
  float4 v[R + 4];
#pragma unroll
  for (int r = 0; r < R + 4; ++r) {
    const v4f_t t = *reinterpret_cast<const GlobalV4f*>(row_base(a.in, r) + x * 4u);
    v[r] = make_float4(t.x, t.y, t.z, t.w);
  }
  const float g0 = a.g0, g1 = a.g1, g2 = a.g2;
  auto vert = [&](float t0, float t1, float t2, float t3, float t4) {
    float acc = g0 * t0;
    acc = fmaf(g1, t1, acc);
    acc = fmaf(g2, t2, acc);
    acc = fmaf(g1, t3, acc);
    return fmaf(g0, t4, acc);
  };
  float4 c[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    c[r] = make_float4(vert(v[r].x, v[r + 1].x, v[r + 2].x, v[r + 3].x, v[r + 4].x),
                       vert(v[r].y, v[r + 1].y, v[r + 2].y, v[r + 3].y, v[r + 4].y),
                       vert(v[r].z, v[r + 1].z, v[r + 2].z, v[r + 3].z, v[r + 4].z),
                       vert(v[r].w, v[r + 1].w, v[r + 2].w, v[r + 3].w, v[r + 4].w));
  if (left_out || right_out) {
    // the outer pair, vertical pass, published by the lane that borders it
    float2* dst = left_out ? &hi[0][0] : &lo[nw + 1][0];
    if (lane == (left_out ? 0 : 63))
#pragma unroll
      for (int r = 0; r < R; ++r)
        dst[r] = make_float2(vert(e0[r], e0[r + 1], e0[r + 2], e0[r + 3], e0[r + 4]),
                             vert(e1[r], e1[r + 1], e1[r + 2], e1[r + 3], e1[r + 4]));
  }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) lo[wave + 1][r] = make_float2(c[r].x, c[r].y);
    if (wave == 0 && bx == 0)  // image border: the clamped columns repeat column 0
#pragma unroll
      for (int r = 0; r < R; ++r) hi[0][r] = make_float2(c[r].x, c[r].x);
  } else if (lane == 63) {
#pragma unroll
    for (int r = 0; r < R; ++r) hi[wave + 1][r] = make_float2(c[r].z, c[r].w);
    if (wave == nw - 1 && bx + 1 == gridDim.x)  // image border: column w - 1 repeated
#pragma unroll
      for (int r = 0; r < R; ++r) lo[nw + 1][r] = make_float2(c[r].w, c[r].w);
  }
  __syncthreads();
  // lane 0 takes the left neighbour's last pair, every other lane the right
  // neighbour's first pair (only lane 63 uses it)
  const float2* halo = lane == 0 ? &hi[wave][0] : &lo[wave + 2][0];
  float2 f[R];
#pragma unroll
  for (int r = 0; r < R; ++r) f[r] = halo[r];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float cc[8] = {from_left(c[r].z, f[r].x), from_left(c[r].w, f[r].y), c[r].x, c[r].y,
                         c[r].z, c[r].w, from_right(c[r].x, f[r].x), from_right(c[r].y, f[r].y)};
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = vert(cc[j], cc[j + 1], cc[j + 2], cc[j + 3], cc[j + 4]);
    const int y = y0 + r;
    if (y < h) {
      uint64_t orow = reinterpret_cast<uint64_t>(a.out) + (uint64_t)(uint32_t)y * pitch;
      asm("" : "+s"(orow));
      __builtin_nontemporal_store(make_v4f(o[0], o[1], o[2], o[3]), reinterpret_cast<GlobalV4f*>(orow + x * 4u));
    }
  }
}

template __global__ void k_gauss5_band_f32<4>(GaussArgs a);
template __global__ void k_gauss5_band_f32<8>(GaussArgs a);
template __global__ void k_gauss5_win_f32<2, true>(GaussArgs a);
template __global__ void k_gauss5_win_f32<4, true>(GaussArgs a);
template __global__ void k_gauss5_win_f32<2, false>(GaussArgs a);
template __global__ void k_gauss5_win_f32<4, false>(GaussArgs a);

// Sobel with the same window, vertical pass first.  The two 3x3 kernels
// factor into a vertical and a horizontal 3-tap pass: gx = horizontal
// difference of the vertical smoothing, gy = horizontal smoothing of the
// vertical difference.  Each lane forms both vertical terms for its 4 columns
// (lanes 0 and 63 also for the column beyond the wave's edge), then takes the
// neighbouring columns' terms by DPP lane shift.  Mask bytes of a lane go out
// as one 4-byte store, and their popcount is the lane's count for the row;
// each wave writes its own (count, sum) partial, so there is no block-wide
// barrier, and the final kernel combines the partials in a fixed order.
template <int R, bool FULL>
__global__ __launch_bounds__(kBlock) void k_sobel_thresh_win_f32(SobelArgs a) {
  unsigned bx, by;
  xcd_tile(bx, by);
  const int w = a.w, h = a.h, wm = w - 1, hm = h - 1;
  const WinLane<FULL> L(w, bx, by, R);
  const int xw = (int)bx * kWinCols;
  const unsigned hx = clampi(L.lane == 0 ? xw - 1 : xw + kWinCols, 0, wm);
  float4 v[R + 2];
  float e[R + 2];
#pragma unroll
  for (int r = 0; r < R + 2; ++r) {
    const float* row = a.blur + (size_t)clampi(L.y0 + r - 1, 0, hm) * w;
    v[r] = L.load4(row);
    e[r] = load1(row, hx);
  }
  const float thr = a.thr;
  float sum = 0.f;
  uint32_t cnt = 0;
  // GUARD: test each row against the image (the last row of blocks, and
  // lanes past a ragged right edge).  Full-width waves whose rows all lie
  // inside take the unguarded copy: their results are used unconditionally,
  // so the compiler keeps every load above this point (one memory round trip)
  // instead of sinking part of a row's load into the row's branch.  Both
  // copies accumulate in the same order.
  auto rows = [&](auto guard) {
    constexpr bool GUARD = decltype(guard)::value;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = L.y0 + r;
      float vs[4], vd[4];  // vertical smoothing (above + 2*centre + below) and difference (below - above)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float t0 = (&v[r].x)[j], t1 = (&v[r + 1].x)[j], t2 = (&v[r + 2].x)[j];
        vs[j] = (t0 + 2.f * t1) + t2;
        vd[j] = t2 - t0;
      }
      const float es = (e[r] + 2.f * e[r + 1]) + e[r + 2], ed = e[r + 2] - e[r];
      const float cs[6] = {from_left(vs[3], es), vs[0], vs[1], vs[2], vs[3], from_right(vs[0], es)};
      const float cd[6] = {from_left(vd[3], ed), vd[0], vd[1], vd[2], vd[3], from_right(vd[0], ed)};
      uint32_t packed = 0;
      float rsum;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float gx = cs[j + 2] - cs[j];
        const float gy = (cd[j] + 2.f * cd[j + 1]) + cd[j + 2];
        const float mag = sqrt_hw(gx * gx + gy * gy);
        packed |= (mag > thr ? 1u : 0u) << (8 * j);
        rsum = (j == 0) ? mag : rsum + mag;
      }
      if (!GUARD || (y < h && !L.past)) {
        uint8_t* mrow = a.mask + (size_t)y * w;  // wave-uniform row base
        store_nt(reinterpret_cast<uint32_t*>(mrow + L.x), packed);
        cnt += __builtin_popcount(packed);
        sum += rsum;
      }
    }
  };
  if (FULL && L.y0 + R <= h)
    rows(std::false_type{});
  else
    rows(std::true_type{});
  const float ws = wave_total_f32(sum);
  const uint32_t wc = wave_total_u32(cnt);
  if (L.lane == 0) {
    const unsigned part = (by * gridDim.x + bx) * 4 + (threadIdx.x >> 6);
    a.psum[part] = ws;
    a.pcount[part] = wc;
  }
}
template __global__ void k_sobel_thresh_win_f32<2, true>(SobelArgs a);
template __global__ void k_sobel_thresh_win_f32<4, true>(SobelArgs a);
template __global__ void k_sobel_thresh_win_f32<2, false>(SobelArgs a);
template __global__ void k_sobel_thresh_win_f32<4, false>(SobelArgs a);

// ------------------------------------------------------------------ thermal grid step
// T' = T + CP*P + CY*(N + S - 2T) + CX*(W + E - 2T) + CZ*(T_AMB - T), a
// neighbour outside the grid being the cell itself.
namespace hotspot {
constexpr float CX = 0.1f, CY = 0.1f, CZ = 1.0f / 640.0f, CP = 0.5f, T_AMB = 300.0f;
__device__ inline float step(float t, float p, float n, float s, float w, float e) {
  const float lap_y = (n + s) - 2.f * t;
  const float lap_x = (w + e) - 2.f * t;
  return t + CP * p + CY * lap_y + CX * lap_x + CZ * (T_AMB - t);
}
}  // namespace hotspot

// Register window as for the image stages: a lane owns 4 columns, a wave 256
// columns x kHotWinRows rows with its rows of T (plus one above and below)
// and of P loaded before the first result.
template <bool FULL>
__global__ __launch_bounds__(kBlock) void k_hotspot_win_f32(HotspotArgs a) {
  constexpr int R = kHotWinRows;
  unsigned bx, by;
  xcd_tile(bx, by);
  if (a.first && bx == 0 && by == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, a.js);
  const int w = a.w, h = a.h, wm = w - 1, hm = h - 1;
  const WinLane<FULL> L(w, bx, by, R);
  const int xw = (int)bx * kWinCols;
  const unsigned hx = clampi(L.lane == 0 ? xw - 1 : xw + kWinCols, 0, wm);
  float4 v[R + 2], pv[R];
  float e[R + 2];
#pragma unroll
  for (int r = 0; r < R + 2; ++r) {
    const float* row = a.tin + (size_t)clampi(L.y0 + r - 1, 0, hm) * w;
    v[r] = L.load4(row);
    e[r] = load1(row, hx);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) pv[r] = L.load4(a.p + (size_t)clampi(L.y0 + r, 0, hm) * w);
  // Full-width waves whose rows all lie inside store unguarded, which keeps
  // every load (P's rows included) above this point: one memory round trip.
  auto rows = [&](auto guard) {
    constexpr bool GUARD = decltype(guard)::value;
#pragma unroll
    for (int r = 1; r <= R; ++r) {
      const int y = L.y0 + r - 1;
      const float c[6] = {from_left(v[r].w, e[r]), v[r].x, v[r].y, v[r].z, v[r].w, from_right(v[r].x, e[r])};
      const float n4[4] = {v[r - 1].x, v[r - 1].y, v[r - 1].z, v[r - 1].w};
      const float s4[4] = {v[r + 1].x, v[r + 1].y, v[r + 1].z, v[r + 1].w};
      const float p4[4] = {pv[r - 1].x, pv[r - 1].y, pv[r - 1].z, pv[r - 1].w};
      float o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] = hotspot::step(c[j + 1], p4[j], n4[j], s4[j], c[j], c[j + 2]);
      if (!GUARD || (y < h && !L.past))
        store_nt(reinterpret_cast<float*>(reinterpret_cast<char*>(a.tout + (size_t)y * w) + L.x * 4u), o[0], o[1],
                 o[2], o[3]);
    }
  };
  if (FULL && L.y0 + R <= h)
    rows(std::false_type{});
  else
    rows(std::true_type{});
}
// Thermal step on row bands, for widths that are a multiple of kBandCols
// and grids of 2^22 to 2^24 cells: 8 waves side by side across R rows (8 up
// to 2^22 cells, 16 above), as the Gaussian's bands.  The halo is
// one raw column each side: lane 0 publishes its first column, lane 63 its
// last, for each of the R rows; after one barrier lanes 0 and 63 read the
// neighbouring waves' columns.  A block's outer columns inside the grid are
// loaded by its first and last wave; at the grid border the neighbour is the
// cell itself.  The per-cell arithmetic is the window kernel's.
template <int R>
__global__ __launch_bounds__(kBandCols / 4) void k_hotspot_band_f32(HotspotArgs a) {
  constexpr int nw = kBandCols / kWinCols;
  unsigned bx, band;
  xcd_tile(bx, band);  // grid (column blocks, bands)
  if (a.first && bx == 0 && band == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, a.js);
  __shared__ float lo[nw + 2][R], hi[nw + 2][R];
  const int w = a.w, h = a.h, hm = h - 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int y0 = (int)band * R;
  const unsigned xb = bx * (unsigned)kBandCols;
  const unsigned x = xb + (unsigned)wave * kWinCols + 4u * (unsigned)lane;
  const uint32_t pitch = (uint32_t)w * 4u;
  const bool left_out = wave == 0 && bx > 0;
  const bool right_out = wave == nw - 1 && bx + 1 < gridDim.x;
  auto row_base = [&](const float* g, int r) {  // row y0 + r, clamped
    uint64_t row = reinterpret_cast<uint64_t>(g) + (uint64_t)(uint32_t)clampi(y0 + r, 0, hm) * pitch;
    asm("" : "+s"(row));
    return row;
  };
  float e[R];
  if (left_out || right_out) {
    const unsigned hc = (left_out ? xb - 1u : xb + (unsigned)kBandCols) * 4u;
#pragma unroll
    for (int r = 0; r < R; ++r) e[r] = *reinterpret_cast<const GlobalF32*>(row_base(a.tin, r) + hc);
  }
  float4 v[R + 2], pv[R];
#pragma unroll
  for (int r = 0; r < R + 2; ++r) {
    const v4f_t t = *reinterpret_cast<const GlobalV4f*>(row_base(a.tin, r - 1) + x * 4u);
    v[r] = make_float4(t.x, t.y, t.z, t.w);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const v4f_t t = *reinterpret_cast<const GlobalV4f*>(row_base(a.p, r) + x * 4u);
    pv[r] = make_float4(t.x, t.y, t.z, t.w);
  }
  if (left_out || right_out) {
    float* dst = left_out ? &hi[0][0] : &lo[nw + 1][0];
    if (lane == (left_out ? 0 : 63))
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r] = e[r];
  }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) lo[wave + 1][r] = v[r + 1].x;
    if (wave == 0 && bx == 0)
#pragma unroll
      for (int r = 0; r < R; ++r) hi[0][r] = v[r + 1].x;
  } else if (lane == 63) {
#pragma unroll
    for (int r = 0; r < R; ++r) hi[wave + 1][r] = v[r + 1].w;
    if (wave == nw - 1 && bx + 1 == gridDim.x)
#pragma unroll
      for (int r = 0; r < R; ++r) lo[nw + 1][r] = v[r + 1].w;
  }
  __syncthreads();
  const float* halo = lane == 0 ? &hi[wave][0] : &lo[wave + 2][0];
  float f[R];
#pragma unroll
  for (int r = 0; r < R; ++r) f[r] = halo[r];
#pragma unroll
  for (int r = 1; r <= R; ++r) {
    const int y = y0 + r - 1;
    const float c[6] = {from_left(v[r].w, f[r - 1]), v[r].x, v[r].y, v[r].z, v[r].w, from_right(v[r].x, f[r - 1])};
    const float n4[4] = {v[r - 1].x, v[r - 1].y, v[r - 1].z, v[r - 1].w};
    const float s4[4] = {v[r + 1].x, v[r + 1].y, v[r + 1].z, v[r + 1].w};
    const float p4[4] = {pv[r - 1].x, pv[r - 1].y, pv[r - 1].z, pv[r - 1].w};
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = hotspot::step(c[j + 1], p4[j], n4[j], s4[j], c[j], c[j + 2]);
    if (y < h) {
      uint64_t orow = reinterpret_cast<uint64_t>(a.tout) + (uint64_t)(uint32_t)y * pitch;
      asm("" : "+s"(orow));
      __builtin_nontemporal_store(make_v4f(o[0], o[1], o[2], o[3]), reinterpret_cast<GlobalV4f*>(orow + x * 4u));
    }
  }
}
template __global__ void k_hotspot_band_f32<8>(HotspotArgs a);
template __global__ void k_hotspot_band_f32<16>(HotspotArgs a);
template __global__ void k_hotspot_win_f32<true>(HotspotArgs a);
template __global__ void k_hotspot_win_f32<false>(HotspotArgs a);

// Widths that are not a multiple of 4: one cell per thread.
__global__ __launch_bounds__(kBlock) void k_hotspot_f32(HotspotArgs a) {
  if (a.first && blockIdx.x == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, a.js);
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (int64_t)a.h * a.w) return;
  const int y = (int)(i / a.w), x = (int)(i - (int64_t)y * a.w);
  const int wm = a.w - 1, hm = a.h - 1;
  const float* T = a.tin;
  const float t = T[i];
  const float n = T[(size_t)clampi(y - 1, 0, hm) * a.w + x], s = T[(size_t)clampi(y + 1, 0, hm) * a.w + x];
  const float wv = T[(size_t)y * a.w + clampi(x - 1, 0, wm)], ev = T[(size_t)y * a.w + clampi(x + 1, 0, wm)];
  a.tout[i] = hotspot::step(t, a.p[i], n, s, wv, ev);
}

// One block: fixed-order combination of the partial counts and sums (one per
// wave on the window path, one per block on the LDS-tile path).
__global__ __launch_bounds__(kBlock) void k_sobel_final(SobelFinalArgs a) {
  __shared__ float s4f[4];
  __shared__ uint32_t s4u[4];
  // Thread t takes 16-byte groups t, t + 256, t + 512, ... (four partials
  // each), four groups per step with independent loads in flight, then the
  // last nparts % 4 partials.  The order depends only on nparts.  Both arrays
  // start 256-byte aligned.
  const float4* ps4 = reinterpret_cast<const float4*>(a.psum);
  const uint4* pc4 = reinterpret_cast<const uint4*>(a.pcount);
  const unsigned n4 = a.nparts >> 2;
  float s = 0.f;
  uint32_t c = 0;
  unsigned k = threadIdx.x;
  for (; k + 3 * kBlock < n4; k += 4 * kBlock) {
    float4 f[4];
    uint4 u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f[i] = ps4[k + i * kBlock];
      u[i] = pc4[k + i * kBlock];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s += (f[i].x + f[i].y) + (f[i].z + f[i].w);
      c += (u[i].x + u[i].y) + (u[i].z + u[i].w);
    }
  }
  for (; k < n4; k += kBlock) {
    const float4 f = ps4[k];
    const uint4 u = pc4[k];
    s += (f.x + f.y) + (f.z + f.w);
    c += (u.x + u.y) + (u.z + u.w);
  }
  const unsigned t = 4 * n4 + threadIdx.x;
  if (t < a.nparts) {
    s += a.psum[t];
    c += a.pcount[t];
  }
  s = block_sum_f32(s, s4f);
  c = block_sum_u32(c, s4u);
  if (threadIdx.x == 0) {
    *a.out_count = c;
    *a.out_sum = s;
    publish_out(a.sc, true);
  }
}

// ------------------------------------------------------------------ vector job: S = sum tanh(a*x + y)
// Block b reduces elements [b*C, min((b+1)*C, n)), C = vec_chunk(n, grid),
// with 16-byte loads when both windows are 4-element aligned.
__global__ __launch_bounds__(kBlock) void k_saxpy_tanh_sum_f32(VecArgs a) {
  __shared__ float s4f[4];
  const JobScalars js = a.js;
  if (blockIdx.x == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, js);
  const uint64_t n = js.n;
  const unsigned G = gridDim.x;
  const uint64_t C = vec_chunk(n, G);
  const uint64_t beg = (uint64_t)blockIdx.x * C;
  const uint64_t end = beg + C < n ? beg + C : n;
  const float* __restrict__ x = a.x + js.x_off;
  const float* __restrict__ y = a.y + js.y_off;
  const float av = js.a;
  float acc = 0.f;
  if (beg < end) {
    if (((js.x_off | js.y_off) & 3u) == 0) {
      const uint64_t vend = beg + ((end - beg) & ~3ull);
      for (uint64_t i = beg + 4ull * threadIdx.x; i < vend; i += 4ull * kBlock) {
        const float4 xv = *reinterpret_cast<const float4*>(x + i);
        const float4 yv = *reinterpret_cast<const float4*>(y + i);
        acc += tanhf(fmaf(av, xv.x, yv.x));
        acc += tanhf(fmaf(av, xv.y, yv.y));
        acc += tanhf(fmaf(av, xv.z, yv.z));
        acc += tanhf(fmaf(av, xv.w, yv.w));
      }
      if (threadIdx.x == 0)
        for (uint64_t i = vend; i < end; ++i) acc += tanhf(fmaf(av, x[i], y[i]));
    } else {
      for (uint64_t i = beg + threadIdx.x; i < end; i += kBlock) acc += tanhf(fmaf(av, x[i], y[i]));
    }
  }
  const float bs = block_sum_f32(acc, s4f);
  if (threadIdx.x == 0) a.partials[blockIdx.x] = bs;
}

// One block: the job's partials (vec_blocks(n) of them) in a fixed order.
// The job's block count comes from n in the slot header.  Every thread loads
// its kVecGridCap / kBlock possible partials beside that load (the scratch
// holds kVecGridCap of them) and adds those below the count, in the order of
// the one-partial-per-step loop: one memory round trip instead of two.
__global__ __launch_bounds__(kBlock) void k_vec_final(VecFinalArgs a) {
  __shared__ float s4f[4];
  static_assert(kVecGridCap % kBlock == 0, "whole partials per thread");
  constexpr int PER = kVecGridCap / kBlock;
  float v[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) v[i] = a.partials[threadIdx.x + i * kBlock];
  const unsigned G = vec_blocks(a.sc.hdr->n);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (threadIdx.x + i * kBlock < G) s += v[i];
  s = block_sum_f32(s, s4f);
  if (threadIdx.x == 0) {
    *a.out_sum = s;
    publish_out(a.sc, true);
  }
}

// ------------------------------------------------------------------ vector batch: persistent (job, tile) kernel
// Every block loops: take the next work item from the batch's counter, find
// its job by binary search over the descriptors' first-item indices, reduce
// that item's elements (fixed order within the item) and store the item's
// partial.  Which block takes which item does not change any result.
template <int BLOCK>
__device__ inline float vec_range_sum(const float* __restrict__ x, const float* __restrict__ y, float av,
                                      uint64_t beg, uint64_t end, bool aligned) {
  float acc = 0.f;
  if (aligned) {
    const uint64_t vend = beg + ((end - beg) & ~3ull);
    for (uint64_t i = beg + 4ull * threadIdx.x; i < vend; i += 4ull * BLOCK) {
      const float4 xv = *reinterpret_cast<const float4*>(x + i);
      const float4 yv = *reinterpret_cast<const float4*>(y + i);
      acc += tanhf(fmaf(av, xv.x, yv.x));
      acc += tanhf(fmaf(av, xv.y, yv.y));
      acc += tanhf(fmaf(av, xv.z, yv.z));
      acc += tanhf(fmaf(av, xv.w, yv.w));
    }
    if (threadIdx.x == 0)
      for (uint64_t i = vend; i < end; ++i) acc += tanhf(fmaf(av, x[i], y[i]));
  } else {
    for (uint64_t i = beg + threadIdx.x; i < end; i += BLOCK) acc += tanhf(fmaf(av, x[i], y[i]));
  }
  return acc;
}

// Pairwise sum of W values in a fixed tree ((s0+s1)+(s2+s3)) + ...
template <int W>
__device__ inline float tree_sum_f32(const float* s) {
  if constexpr (W == 1) {
    return s[0];
  } else {
    return tree_sum_f32<W / 2>(s) + tree_sum_f32<W / 2>(s + W / 2);
  }
}

// Block sum of a BLOCK-thread block: wave sums, then a fixed pairwise tree
// over the waves (for 256 threads the same order as block_sum_f32).
template <int BLOCK>
__device__ inline float block_sum_f32_w(float v, float* sw) {
  v = wave_sum_f32(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sw[wave] = v;
  __syncthreads();
  return tree_sum_f32<BLOCK / 64>(sw);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_vec_batch_tiles(VecBatchArgs a) {
  __shared__ float s4f[BLOCK / 64];
  __shared__ uint32_t s_item;
  __shared__ uint32_t s_job;
  if (blockIdx.x == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, a.js);
  const VecBatchHdr* H = reinterpret_cast<const VecBatchHdr*>(a.tab);
  const VecBatchDesc* D = reinterpret_cast<const VecBatchDesc*>(a.tab + sizeof(VecBatchHdr));
  const uint32_t count = H->count, T = H->total_tiles;
  while (true) {
    if (threadIdx.x == 0) {
      const uint32_t t = __hip_atomic_fetch_add(a.work, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_item = t;
      if (t < T) {
        uint32_t lo = 0, hi = count - 1;
        while (lo < hi) {
          const uint32_t mid = (lo + hi + 1) >> 1;
          if (D[mid].tile_start <= t) lo = mid; else hi = mid - 1;
        }
        s_job = lo;
      }
    }
    __syncthreads();
    const uint32_t t = s_item;
    if (t >= T) break;
    const VecBatchDesc d = D[s_job];
    const uint64_t beg = (uint64_t)(t - d.tile_start) * d.tile_elems;
    const uint64_t end = beg + d.tile_elems < d.n ? beg + d.tile_elems : (uint64_t)d.n;
    const float acc =
        vec_range_sum<BLOCK>(a.x + d.x_off, a.y + d.y_off, d.a, beg, end, ((d.x_off | d.y_off) & 3u) == 0);
    const float bs = block_sum_f32_w<BLOCK>(acc, s4f);
    if (threadIdx.x == 0) a.partials[t] = bs;
    __syncthreads();
  }
}
template __global__ void k_vec_batch_tiles<128>(VecBatchArgs);
template __global__ void k_vec_batch_tiles<256>(VecBatchArgs);
template __global__ void k_vec_batch_tiles<512>(VecBatchArgs);
template __global__ void k_vec_batch_tiles<1024>(VecBatchArgs);

// Job j = thread: its items' partials added in item order.  Block 0 also
// rewinds the work counter for the slot's next batch and publishes the header.
__global__ __launch_bounds__(kBlock) void k_vec_batch_final(VecBatchFinalArgs a) {
  const VecBatchHdr* H = reinterpret_cast<const VecBatchHdr*>(a.tab);
  const VecBatchDesc* D = reinterpret_cast<const VecBatchDesc*>(a.tab + sizeof(VecBatchHdr));
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < H->count) {
    const VecBatchDesc d = D[j];
    a.results[j] = vec_items_total(a.partials, d.tile_start, d.ntiles);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *a.work = 0u;
    publish_out(a.sc, true);
  }
}

// ------------------------------------------------------------------ inclusive scan int32 -> int64
// Reduce-then-scan: tile sums, an exclusive scan of the tile sums in one
// block, then each tile scans itself from its offset.  Integer addition is
// exact, so any order gives the same sums; no block waits on another.

// Loads the kScanItems values thread tid owns in tile t (zeros past n).
__device__ inline void scan_load(const int32_t* in, uint64_t n, unsigned t, int tid, int64_t v[kScanItems]) {
  const uint64_t base = (uint64_t)t * kScanTile + (uint64_t)tid * kScanItems;
  if (base + kScanItems <= n) {
    const int4 p0 = *reinterpret_cast<const int4*>(in + base);
    const int4 p1 = *reinterpret_cast<const int4*>(in + base + 4);
    v[0] = p0.x; v[1] = p0.y; v[2] = p0.z; v[3] = p0.w;
    v[4] = p1.x; v[5] = p1.y; v[6] = p1.z; v[7] = p1.w;
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? (int64_t)in[base + k] : 0;
  }
}

// One DPP move of a 64-bit value (both halves): lanes whose source lies
// outside their row, or whose row or bank the masks leave out, read 0.
template <int CTRL, int ROWS, int BANKS>
__device__ inline int64_t dpp_i64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, BANKS, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, BANKS, false);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Inclusive scan of one int64 per lane over the wave, in registers: adding
// the input shifted right by 1, 2 and 3 lanes gives each lane the sum of its
// 4-lane window; row_shr:4 into banks 1-3 and row_shr:8 into banks 2-3 extend
// that to the lane's prefix of its 16-lane row; row_bcast:15 into rows 1 and
// 3 and row_bcast:31 into rows 2 and 3 add the totals of the rows below.
__device__ inline int64_t wave_inclusive_i64(int64_t x) {
  int64_t v = x;
  v += dpp_i64<0x111, 0xf, 0xf>(x);  // row_shr:1
  v += dpp_i64<0x112, 0xf, 0xf>(x);  // row_shr:2
  v += dpp_i64<0x113, 0xf, 0xf>(x);  // row_shr:3
  v += dpp_i64<0x114, 0xf, 0xe>(v);  // row_shr:4
  v += dpp_i64<0x118, 0xf, 0xc>(v);  // row_shr:8
  v += dpp_i64<0x142, 0xa, 0xf>(v);  // row_bcast:15
  v += dpp_i64<0x143, 0xc, 0xf>(v);  // row_bcast:31
  return v;
}

// Exclusive block scan of one int64 per thread; returns the thread's exclusive
// prefix and the block total.
__device__ inline int64_t block_exclusive_i64(int64_t x, int64_t* s_wave, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t inc = wave_inclusive_i64(x);
  __syncthreads();
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  int64_t wave_excl = 0;
  for (int i = 0; i < wave; ++i) wave_excl += s_wave[i];
  *total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
  return wave_excl + inc - x;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce_i32(ScanReduceArgs a) {
  __shared__ int64_t s_wave[4];
  const JobScalars js = a.js;
  const unsigned t = blockIdx.x;
  if (t == 0 && threadIdx.x == 0) write_slot_hdr(a.hdr, js);
  if ((uint64_t)t * kScanTile >= js.n) return;
  int64_t v[kScanItems];
  scan_load(a.in, js.n, t, threadIdx.x, v);
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) s += v[k];
  int64_t total;
  block_exclusive_i64(s, s_wave, &total);
  if (threadIdx.x == 0) a.tile_sum[t] = total;
}

// A thread's 8 tile sums are four 16-byte loads with no branch around them:
// past the last tile it re-reads the last 8-sum group (inside the scratch,
// which is padded to 256 bytes) and drops what lies beyond.
__global__ __launch_bounds__(kBlock) void k_scan_spine_i64(ScanSpineArgs a) {
  __shared__ int64_t s_wave[4];
  const unsigned T = scan_tiles(a.n);
  const unsigned last = (T - 1) & ~(unsigned)(kScanItems - 1);
  int64_t carry = 0;
  for (unsigned base = 0; base < T; base += kScanTile) {
    int64_t v[kScanItems];
    const unsigned i0 = base + threadIdx.x * kScanItems;
    const longlong2* g = reinterpret_cast<const longlong2*>(a.tile_sum + (i0 < last ? i0 : last));
#pragma unroll
    for (int q = 0; q < kScanItems / 2; ++q) {
      const longlong2 t = g[q];
      v[2 * q] = t.x;
      v[2 * q + 1] = t.y;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = (i0 + k < T) ? v[k] : 0;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    int64_t total;
    const int64_t ex = block_exclusive_i64(s, s_wave, &total);
    int64_t run = carry + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (i0 + k < T) a.tile_excl[i0 + k] = run;
      run += v[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) publish_out(a.sc, true);
}

// Results are computed in the blocked order the loads use (8 consecutive
// elements per thread), then pass through LDS so that each store instruction
// of a wave writes one contiguous 1 KiB run: a thread's own 64-byte run would
// make every store instruction touch 32 lines a quarter each.
__global__ __launch_bounds__(kBlock) void k_scan_down_i32_i64(ScanDownArgs a) {
  constexpr int kPitch = kScanItems + 2;  // LDS row of a thread (padding spreads the banks, keeps 16-byte alignment)
  __shared__ int64_t s_wave[4];
  __shared__ __align__(16) int64_t s_out[kBlock * kPitch];
  const uint64_t n = a.n;
  const unsigned t = blockIdx.x;
  if ((uint64_t)t * kScanTile >= n) return;
  // The thread's 8 values as two 16-byte loads with no branch around them,
  // then the tile's prefix, held at this point by the empty asm statement
  // (the compiler would otherwise load it after the block scan, or after
  // waiting for the data behind a branch: a second memory round trip).  So
  // one memory latency covers both.  A thread past the end reads the last
  // 8-value group instead and zeroes what lies beyond n: the slot's input
  // region is padded to 256 bytes, so a 32-byte group that starts below n
  // lies inside it.
  const uint64_t base = (uint64_t)t * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  const uint64_t last = (n - 1) & ~(uint64_t)(kScanItems - 1);
  const uint64_t ld = base < last ? base : last;
  const int4 q0 = *reinterpret_cast<const int4*>(a.in + ld);
  const int4 q1 = *reinterpret_cast<const int4*>(a.in + ld + 4);
  const int64_t tile_off = a.tile_excl[t];
  asm volatile("" ::"s"(tile_off) : "memory");
  int64_t v[kScanItems] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? v[k] : 0;
#pragma unroll
  for (int k = 1; k < kScanItems; ++k) v[k] += v[k - 1];
  int64_t total;
  const int64_t off0 = tile_off + block_exclusive_i64(v[kScanItems - 1], s_wave, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) s_out[threadIdx.x * kPitch + k] = off0 + v[k];
  __syncthreads();
  const uint64_t tile0 = (uint64_t)t * kScanTile;
  auto at = [&](int e) { return s_out[(e / kScanItems) * kPitch + (e % kScanItems)]; };
  if (!a.low32) {
    int64_t* o = reinterpret_cast<int64_t*>(a.out) + tile0;
    if (tile0 + kScanTile <= n) {
#pragma unroll
      for (int k = 0; k < kScanItems / 2; ++k) {
        const int e = 2 * (k * kBlock + (int)threadIdx.x);  // element pairs in striped order
        store_nt(o + e, at(e), at(e + 1));
      }
    } else {
      for (int e = threadIdx.x; e < kScanTile; e += kBlock)
        if (tile0 + e < n) o[e] = at(e);
    }
  } else {
    uint32_t* o = reinterpret_cast<uint32_t*>(a.out) + tile0;
    if (tile0 + kScanTile <= n) {
#pragma unroll
      for (int k = 0; k < kScanItems / 4; ++k) {
        const int e = 4 * (k * kBlock + (int)threadIdx.x);  // element quads in striped order
        store_nt(o + e, (uint32_t)at(e), (uint32_t)at(e + 1), (uint32_t)at(e + 2), (uint32_t)at(e + 3));
      }
    } else {
      for (int e = threadIdx.x; e < kScanTile; e += kBlock)
        if (tile0 + e < n) o[e] = (uint32_t)at(e);
    }
  }
}

}  // namespace setrt
