// Tile geometry and grid sizes of the stage kernels.  Plain C++ so host-only
// code (slot layout, scheduler, fake backend) shares it without HIP headers.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define SETRT_HD __host__ __device__
#else
#define SETRT_HD
#endif

namespace setrt {

constexpr int kBlock = 256;
constexpr int kBoxTW = 64, kBoxTH = 16;       // 3x3 box: output tile
constexpr int kDivPerThread = 8;              // floor(s/9): pixels per thread
constexpr int kHistPerThread = 16;            // histogram: pixels per thread
constexpr int kGaussTW = 64, kGaussTH = 16;   // separable Gaussian: output tile
constexpr int kSobelTW = 64, kSobelTH = 16;   // Sobel: output tile
constexpr int kVecChunk = 2048;               // vector job: elements per block (multiple of 4*kBlock)
constexpr int kVecGridCap = 2048;             // vector job: most blocks per job
constexpr int kScanItems = 8;                 // scan: items per thread
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kCopyBlocks = 32;               // host<->device copy kernels: small grid, PCIe-bound
// Device-to-host copies of 1 MiB and more take 64 blocks: with a host-to-device
// pull running beside them, 32 + 64 blocks moved 67 GB/s in both directions
// together against 57 GB/s for 32 + 32.
inline unsigned d2h_copy_blocks(uint64_t bytes) { return bytes >= (1ull << 20) ? 64u : (unsigned)kCopyBlocks; }
constexpr int kVecBatchGrid = 1024;           // persistent vector-batch kernel: default grid

// Default work-item size for vector jobs of size bucket b = floor(log2 n):
// about eight items per job, a multiple of 1024 elements, within [1024, 65536].
inline uint32_t vec_default_tile(int b) {
  uint64_t t = (b >= 3) ? (1ull << (b - 3)) : 1ull;
  t = (t + 1023) / 1024 * 1024;
  if (t < 1024) t = 1024;
  if (t > 65536) t = 65536;
  return (uint32_t)t;
}

struct Grid3 {
  unsigned x, y, z;
};

inline Grid3 box_grid(int h, int w) {
  return {(unsigned)((w + kBoxTW - 1) / kBoxTW), (unsigned)((h + kBoxTH - 1) / kBoxTH), 1u};
}
inline unsigned div9_blocks(int64_t npix) {
  return (unsigned)((npix + (int64_t)kBlock * kDivPerThread - 1) / ((int64_t)kBlock * kDivPerThread));
}
inline unsigned hist_blocks(int64_t npix) {
  return (unsigned)((npix + (int64_t)kBlock * kHistPerThread - 1) / ((int64_t)kBlock * kHistPerThread));
}
// Float images whose width is a multiple of 4 take the register-window
// kernels: a lane owns 4 adjacent columns (16-byte loads and stores), a wave
// 256 columns x R rows, a block 4 waves stacked vertically.  The Gaussian
// takes R = 2 below 1024^2 pixels and Sobel up to 1024^2, both R = 4 above
// (more blocks in flight pay on the smaller images, fewer re-read halo rows on
// the larger).  Other widths take the LDS-tile kernels.  The Gaussian of
// widths that are multiples of kBandCols takes the row-band kernel instead.
constexpr int kWinCols = 256;                 // columns per wave (and per block)
// Gaussian row bands for widths that are a multiple of kBandCols: blocks of
// 8 waves side by side (2048 columns) across R rows, R = 8 up to 4096^2
// pixels and 4 above.  Measured on cold buffers (window kernel / band R = 4 /
// band R = 8): 8.6 / 8.1 / 7.2 us at 2048^2, 29.2 / 28.3 / 28.0 us at 4096^2,
// 99.7 / 92.4 / 94.3 us at 8192^2.  At 1024^2 (blocks of 4 waves across the
// width) a 4-row band was the slower, 3.7 against 3.6 us, and 16-wave blocks
// across 4096 columns took 31 us.
constexpr int kBandCols = 2048;
inline bool gauss_band_path(int w) { return w > 0 && (w % kBandCols) == 0; }
inline int gauss_band_rows(int h, int w) { return (int64_t)h * w <= (int64_t)4096 * 4096 ? 8 : 4; }
inline bool image_window_path(int w) { return w > 0 && (w % 4) == 0; }
// Every tile of the window path full width: no lane lies past the right edge.
inline bool window_full_width(int w) { return w > 0 && (w % kWinCols) == 0; }
inline int gauss_win_rows(int h, int w) { return (int64_t)h * w < (int64_t)1024 * 1024 ? 2 : 4; }
inline int sobel_win_rows(int h, int w) { return (int64_t)h * w <= (int64_t)1024 * 1024 ? 2 : 4; }
inline Grid3 window_grid(int h, int w, int rows_per_wave) {
  const int rows = 4 * rows_per_wave;
  return {(unsigned)((w + kWinCols - 1) / kWinCols), (unsigned)((h + rows - 1) / rows), 1u};
}
inline Grid3 gauss_grid(int h, int w) {
  if (gauss_band_path(w)) {
    const int r = gauss_band_rows(h, w);
    return {(unsigned)(w / kBandCols), (unsigned)((h + r - 1) / r), 1u};
  }
  if (image_window_path(w)) return window_grid(h, w, gauss_win_rows(h, w));
  return {(unsigned)((w + kGaussTW - 1) / kGaussTW), (unsigned)((h + kGaussTH - 1) / kGaussTH), 1u};
}
inline Grid3 sobel_grid(int h, int w) {
  if (image_window_path(w)) return window_grid(h, w, sobel_win_rows(h, w));
  return {(unsigned)((w + kSobelTW - 1) / kSobelTW), (unsigned)((h + kSobelTH - 1) / kSobelTH), 1u};
}
// Sobel's partial (count, sum) pairs: one per wave on the window path, one per
// block on the LDS-tile path.
inline uint64_t sobel_partials(int h, int w) {
  const Grid3 g = sobel_grid(h, w);
  return (uint64_t)g.x * g.y * (image_window_path(w) ? 4u : 1u);
}
// Thermal-grid step: the register window (4 columns x kHotWinRows rows per
// lane) for widths that are multiples of 4, one pixel per thread otherwise.
constexpr int kHotWinRows = 2;
// Row bands (the Gaussian's layout) for widths that are a multiple of
// kBandCols and grids of 2^22 to 2^24 cells: 8 rows per band up to 2^22
// cells, 16 above; 0 = not the band path.  Measured cold per step (window /
// 8-row / 16-row band): 10.3 / 9.0 / 10.4 us at 2048^2, 10.3 / 9.4 us at
// 4096x1024, 38.9 / 39.6 / 37.4 us at 4096^2; at 2048x1024 the 8-row band
// was the slower (6.9 against 6.1 us).
inline int hotspot_band_rows(int h, int w) {
  const int64_t n = (int64_t)h * w;
  if (w <= 0 || (w % kBandCols) != 0 || n < ((int64_t)1 << 22) || n > ((int64_t)1 << 24)) return 0;
  return n <= ((int64_t)1 << 22) ? 8 : 16;
}
inline Grid3 hotspot_grid(int h, int w) {
  if (const int r = hotspot_band_rows(h, w)) return {(unsigned)(w / kBandCols), (unsigned)((h + r - 1) / r), 1u};
  if (image_window_path(w)) return window_grid(h, w, kHotWinRows);
  const uint64_t n = (uint64_t)h * w;
  return {(unsigned)((n + kBlock - 1) / kBlock), 1u, 1u};
}
// Vector job: blocks for length n.  Deterministic in n, so the reduction
// order of a job depends only on its length.
SETRT_HD inline unsigned vec_blocks(uint64_t n) {
  uint64_t b = (n + kVecChunk - 1) / kVecChunk;
  if (b < 1) b = 1;
  if (b > (uint64_t)kVecGridCap) b = kVecGridCap;
  return (unsigned)b;
}
// Elements per block for length n over g blocks (a multiple of 4*kBlock).
SETRT_HD inline uint64_t vec_chunk(uint64_t n, unsigned g) {
  uint64_t c = (n + g - 1) / g;
  const uint64_t q = 4ull * kBlock;
  return (c + q - 1) / q * q;
}
SETRT_HD inline unsigned scan_tiles(uint64_t n) { return (unsigned)((n + kScanTile - 1) / kScanTile); }

// Byte layout of one buffer slot of a template (offsets from the slot base,
// all 256-byte aligned).  In debug templates the intermediate images live
// inside the output block so the D2H copy returns them.
struct SlotLayout {
  uint64_t hdr;        // DevSlotHdr
  uint64_t in;         // H2D destination
  uint64_t in_cap;
  uint64_t out;        // output block: set_out_header + payload (+ debug images)
  uint64_t out_cap;
  uint64_t b1, b2;     // intermediates (box: S, Q; gauss: blur, mask)
  uint64_t scratch;    // partials, counters, tile states
  uint64_t scratch_bytes;
  uint64_t tail;       // tail canary
  uint64_t total;
};

}  // namespace setrt
