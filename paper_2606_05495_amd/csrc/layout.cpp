// Slot layouts, per-job copy sizes and argument validation of every pipeline.
// Host-only, no HIP headers.
#include <cstdio>
#include <string>

#include "internal.hpp"
#include "tiles.hpp"

namespace setrt {

namespace {
constexpr uint64_t kAlign = 256;
inline uint64_t up(uint64_t v, uint64_t a = kAlign) { return (v + a - 1) / a * a; }
}  // namespace

int pipeline_validate(const set_job_template& t, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return SET_EINVAL;
  };
  switch (t.pipeline) {
    case SET_PIPE_BOX_HIST_U8:
    case SET_PIPE_GAUSS_SOBEL_F32:
      if (t.width < 1 || t.height < 1) return bad("image templates need width >= 1 and height >= 1");
      if ((uint64_t)t.width * t.height > (1ull << 28)) return bad("image larger than 2^28 pixels");
      if (t.width > (1u << 20)) return bad("image width larger than 2^20");
      // keeps every image grid within the launch limit of 65,536 blocks in
      // its second dimension: 8 or more rows per block, except the
      // Gaussian's 4-row bands, whose widths of 2048 or more leave at most
      // 2^17 rows
      if (t.height > (1u << 19)) return bad("image height larger than 2^19");
      break;
    case SET_PIPE_SAXPY_TANH_SUM_F32:
      if (t.max_n < 1 || t.max_n > (1ull << 32)) return bad("vector template needs 1 <= max_n <= 2^32");
      if (t.dev_x_pool == nullptr || t.dev_y_pool == nullptr || t.pool_len < 1)
        return bad("vector template needs device x/y pools");
      break;
    case SET_PIPE_SCAN_I32_I64:
      if (t.max_n < 1 || t.max_n > (1ull << 31)) return bad("scan template needs 1 <= max_n <= 2^31");
      break;
    case SET_PIPE_HOTSPOT_F32:
      if (t.width < 1 || t.height < 1) return bad("thermal-grid templates need width >= 1 and height >= 1");
      if ((uint64_t)t.width * t.height > (1ull << 28)) return bad("grid larger than 2^28 cells");
      if (t.width > (1u << 20)) return bad("grid width larger than 2^20");
      if (t.height > (1u << 19)) return bad("grid height larger than 2^19");  // 8 rows per block, as above
      if (t.max_n < 1 || t.max_n > (uint64_t)kMaxHotspotSteps) return bad("thermal-grid template needs 1 <= max_n (steps) <= 32");
      break;
    case SET_PIPE_SCAN_LIB_I32_I64:
      if (t.max_n < 1 || t.max_n > (1ull << 31)) return bad("scan template needs 1 <= max_n <= 2^31");
      if (t.flags & SET_TF_SCAN_LOW32) return bad("the library scan template writes the full int64 output");
      break;
    case SET_PIPE_SAXPY_BATCH_F32:
      if (t.max_n < 1 || t.max_n > (1ull << 32) - 1) return bad("vector batch template needs 1 <= max_n < 2^32");
      if (t.dev_x_pool == nullptr || t.dev_y_pool == nullptr || t.pool_len < 1)
        return bad("vector batch template needs device x/y pools");
      if (t.batch_max < 1 || t.batch_max > (1u << 20)) return bad("vector batch template needs 1 <= batch_max <= 2^20");
      if (t.tiles_max < t.batch_max || t.tiles_max > (1u << 26)) return bad("vector batch needs batch_max <= tiles_max <= 2^26");
      if (t.block != 0 && t.block != 128 && t.block != 256 && t.block != 512 && t.block != 1024)
        return bad("vector batch block must be 0, 128, 256, 512 or 1024");
      break;
    default:
      return bad("unknown pipeline");
  }
  if (t.block != 0 && t.pipeline != SET_PIPE_SAXPY_BATCH_F32)
    return bad("only the vector batch template takes a block size (block must be 0)");
  if (t.flags & ~(uint32_t)(SET_TF_DEBUG | SET_TF_SCAN_LOW32 | SET_TF_CAPTURE | SET_TF_POISON))
    return bad("unknown template flags");
  if (t.stress_delay_us > 100000) return bad("stress_delay_us above 100000");
  if (t.reserved != 0) return bad("reserved template field must be 0");
  if (t.copy_mode != SET_COPY_KERNELS && t.copy_mode != SET_COPY_NODES && t.copy_mode != SET_COPY_ASYNC_IN)
    return bad("unknown copy mode");
  return SET_OK;
}

static SlotLayout layout_of(const set_job_template& t) {
  SlotLayout L{};
  const bool dbg = (t.flags & SET_TF_DEBUG) != 0;
  uint64_t off = 0;
  L.hdr = 0;
  off = up(sizeof(DevSlotHdr));
  switch (t.pipeline) {
    case SET_PIPE_BOX_HIST_U8: {
      const uint64_t npix = (uint64_t)t.width * t.height;
      L.in = off;
      L.in_cap = npix;
      off = up(off + npix);
      L.out = off;
      uint64_t o = 64 + 1024;  // header + uint32 histogram
      if (dbg) {
        const uint64_t s_off = up(o, 64);
        const uint64_t q_off = up(s_off + 2 * npix, 64);
        L.b1 = L.out + s_off;
        L.b2 = L.out + q_off;
        o = q_off + npix;
      }
      L.out_cap = o;
      off = up(off + o);
      if (!dbg) {
        L.b1 = off;
        off = up(off + 2 * npix);
        L.b2 = off;
        off = up(off + npix);
      }
      L.scratch = off;
      L.scratch_bytes = up((uint64_t)hist_blocks((int64_t)npix) * 256 * 4);  // per-block partial histograms
      off = up(off + L.scratch_bytes);
      break;
    }
    case SET_PIPE_GAUSS_SOBEL_F32: {
      const uint64_t npix = (uint64_t)t.width * t.height;
      L.in = off;
      L.in_cap = 4 * npix;
      off = up(off + 4 * npix);
      L.out = off;
      uint64_t o = 64 + 8;  // header + {count, sum}
      if (dbg) {
        const uint64_t m_off = 128;
        const uint64_t b_off = up(m_off + npix, 64);
        L.b2 = L.out + m_off;  // mask
        L.b1 = L.out + b_off;  // blur
        o = b_off + 4 * npix;
      }
      L.out_cap = o;
      off = up(off + o);
      if (!dbg) {
        L.b1 = off;
        off = up(off + 4 * npix);
        L.b2 = off;
        off = up(off + npix);
      }
      const uint64_t nb = sobel_partials((int)t.height, (int)t.width);
      L.scratch = off;
      L.scratch_bytes = up(nb * 4) + up(nb * 4);  // partial counts, partial sums
      off = up(off + L.scratch_bytes);
      break;
    }
    case SET_PIPE_SAXPY_TANH_SUM_F32: {
      L.in = off;
      L.in_cap = 0;
      L.out = off;
      L.out_cap = 64 + 4;
      off = up(off + L.out_cap);
      L.scratch = off;
      L.scratch_bytes = up((uint64_t)kVecGridCap * 4);  // per-block partial sums
      off = up(off + L.scratch_bytes);
      break;
    }
    case SET_PIPE_SAXPY_BATCH_F32: {
      L.in = off;
      L.in_cap = 64 + 48ull * t.batch_max;
      off = up(off + L.in_cap);
      L.out = off;
      L.out_cap = 64 + 4ull * t.batch_max;
      off = up(off + L.out_cap);
      L.scratch = off;
      L.scratch_bytes = up(4ull * t.tiles_max) + kAlign;  // per-work-item partials, work counter
      off = up(off + L.scratch_bytes);
      break;
    }
    case SET_PIPE_HOTSPOT_F32: {
      const uint64_t npix = (uint64_t)t.width * t.height;
      L.in = off;  // T0 then P
      L.in_cap = 8 * npix;
      off = up(off + 8 * npix);
      L.out = off;  // header + T_K
      L.out_cap = 64 + 4 * npix;
      off = up(off + L.out_cap);
      L.b1 = off;  // ping-pong buffers of the intermediate steps
      off = up(off + 4 * npix);
      L.b2 = off;
      off = up(off + 4 * npix);
      L.scratch = off;
      L.scratch_bytes = 0;
      break;
    }
    case SET_PIPE_SCAN_LIB_I32_I64: {
      // the library's temporary storage is a separate per-slot workspace
      const uint64_t n = t.max_n;
      L.in = off;
      L.in_cap = 4 * n;
      off = up(off + 4 * n);
      L.out = off;
      L.out_cap = 64 + 8 * n;
      off = up(off + L.out_cap);
      L.scratch = off;
      L.scratch_bytes = 0;
      break;
    }
    case SET_PIPE_SCAN_I32_I64: {
      const uint64_t n = t.max_n;
      const uint64_t tiles = scan_tiles(n);
      L.in = off;
      L.in_cap = 4 * n;
      off = up(off + 4 * n);
      L.out = off;
      L.out_cap = 64 + ((t.flags & SET_TF_SCAN_LOW32) ? 4 * n : 8 * n);
      off = up(off + L.out_cap);
      L.scratch = off;
      L.scratch_bytes = up(tiles * 8) + up(tiles * 8);  // tile sums, exclusive tile offsets
      off = up(off + L.scratch_bytes);
      break;
    }
    default:
      break;
  }
  L.tail = off;
  off = up(off + 8);
  L.total = off;
  return L;
}

SlotLayout slot_layout(const set_job_template& t) { return layout_of(t); }

uint64_t pipeline_in_bytes(const set_job_template& t, uint64_t n) {
  switch (t.pipeline) {
    case SET_PIPE_BOX_HIST_U8:
      return (uint64_t)t.width * t.height;
    case SET_PIPE_GAUSS_SOBEL_F32:
      return 4ull * t.width * t.height;
    case SET_PIPE_HOTSPOT_F32:
      return 8ull * t.width * t.height;
    case SET_PIPE_SAXPY_TANH_SUM_F32:
      return 0;
    case SET_PIPE_SCAN_I32_I64:
    case SET_PIPE_SCAN_LIB_I32_I64:
      return 4ull * (n ? n : t.max_n);
    case SET_PIPE_SAXPY_BATCH_F32:
      return 64 + 48ull * n;
  }
  return 0;
}

uint64_t pipeline_out_bytes(const set_job_template& t, uint64_t n) {
  switch (t.pipeline) {
    case SET_PIPE_BOX_HIST_U8:
    case SET_PIPE_GAUSS_SOBEL_F32:
      return layout_of(t).out_cap;
    case SET_PIPE_SAXPY_TANH_SUM_F32:
      return 64 + 4;
    case SET_PIPE_SCAN_I32_I64:
      return 64 + ((t.flags & SET_TF_SCAN_LOW32) ? 4ull : 8ull) * (n ? n : t.max_n);
    case SET_PIPE_SCAN_LIB_I32_I64:
      return 64 + 8ull * t.max_n;
    case SET_PIPE_HOTSPOT_F32:
      return 64 + 4ull * t.width * t.height;
    case SET_PIPE_SAXPY_BATCH_F32:
      return 64 + 4ull * n;
  }
  return 0;
}

int pipeline_validate_job(const set_job_template& t, const set_job_args& a, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return SET_EINVAL;
  };
  uint64_t n = a.n;
  if (t.pipeline == SET_PIPE_SAXPY_TANH_SUM_F32) {
    if (n < 1 || n > t.max_n) return bad("vector job needs 1 <= n <= template max_n");
    if (a.x_off > t.pool_len || n > t.pool_len - a.x_off) return bad("x window outside the pool");
    if (a.y_off > t.pool_len || n > t.pool_len - a.y_off) return bad("y window outside the pool");
  }
  if (t.pipeline == SET_PIPE_SCAN_I32_I64) {
    if (n == 0) n = t.max_n;
    if (n > t.max_n) return bad("scan job n exceeds template max_n");
  }
  if (t.pipeline == SET_PIPE_SCAN_LIB_I32_I64) {
    if (n == 0) n = t.max_n;
    if (n != t.max_n) return bad("library scan jobs have n = template max_n (the captured call has a fixed length)");
  }
  if (t.pipeline == SET_PIPE_SAXPY_BATCH_F32 && (n < 1 || n > t.batch_max))
    return bad("vector batch job needs 1 <= n (jobs in the batch) <= batch_max");
  const uint64_t ib = pipeline_in_bytes(t, n), ob = pipeline_out_bytes(t, n);
  if (ib > 0 && (a.host_in == nullptr || a.in_bytes != ib)) return bad("host_in missing or in_bytes mismatch");
  if (a.host_out == nullptr || a.out_bytes < ob) return bad("host_out missing or out_bytes too small");
  if (t.copy_mode != SET_COPY_NODES && ((((uintptr_t)a.host_in) | ((uintptr_t)a.host_out)) & 15u))
    return bad("copy kernels need 16-byte aligned host buffers");
  return SET_OK;
}

int pipeline_sizes(const set_job_template& t, TemplateSizes* out) {
  std::string why;
  if (pipeline_validate(t, &why) != SET_OK) return SET_EINVAL;
  const SlotLayout L = layout_of(t);
  TemplateSizes s{};
  s.slot_bytes = L.total;
  auto stage = [&](const char* name, uint64_t bytes) {
    snprintf(s.stage_names[s.num_stages], sizeof(s.stage_names[0]), "%s", name);
    s.stage_bytes[s.num_stages++] = bytes;
  };
  const uint64_t npix = (uint64_t)t.width * t.height;
  switch (t.pipeline) {
    case SET_PIPE_BOX_HIST_U8: {
      const uint64_t hb = hist_blocks((int64_t)npix);
      stage("box3_u8_u16", npix + 2 * npix);
      stage("div9_u16_u8", 2 * npix + npix);
      stage("hist256_u8", npix + hb * 1024);
      stage("hist256_final", hb * 1024 + 1024 + 64);
      break;
    }
    case SET_PIPE_GAUSS_SOBEL_F32: {
      const uint64_t nb = sobel_partials((int)t.height, (int)t.width);
      stage("gauss5_f32", 4 * npix + 4 * npix);
      stage("sobel_thresh_f32", 4 * npix + npix + 8 * nb);
      stage("sobel_final", 8 * nb + 8 + 64);
      break;
    }
    case SET_PIPE_SAXPY_TANH_SUM_F32: {
      const uint64_t G = vec_blocks(t.max_n);
      stage("saxpy_tanh_sum_f32", 8 * t.max_n + 4 * G);
      stage("vec_final", 4 * G + 4 + 64);
      break;
    }
    case SET_PIPE_SAXPY_BATCH_F32:
      // the streamed bytes depend on the batch (8 bytes per element of every job)
      stage("vec_batch_tiles", 64 + 48ull * t.batch_max + 4ull * t.tiles_max);
      stage("vec_batch_final", 64 + 48ull * t.batch_max + 4ull * t.tiles_max + 4ull * t.batch_max);
      break;
    case SET_PIPE_HOTSPOT_F32:
      // each step reads T and P and writes T'
      for (uint64_t k = 0; k < t.max_n; ++k) stage("hotspot_step_f32", 12 * npix);
      stage("job_end", 64 + 64);
      break;
    case SET_PIPE_SCAN_LIB_I32_I64:
      stage("job_begin", 64);
      stage("scan_lib_rocprim", 4 * t.max_n + 8 * t.max_n);  // the library's own traffic is its business
      stage("job_end", 64 + 64);
      break;
    case SET_PIPE_SCAN_I32_I64: {
      const uint64_t T = scan_tiles(t.max_n);
      const uint64_t ob = ((t.flags & SET_TF_SCAN_LOW32) ? 4 : 8) * t.max_n;
      stage("scan_reduce_i32", 4 * t.max_n + 8 * T);
      stage("scan_spine_i64", 16 * T + 64);
      stage("scan_down_i32_i64", 4 * t.max_n + 8 * T + ob);
      break;
    }
  }
  *out = s;
  return SET_OK;
}

}  // namespace setrt
