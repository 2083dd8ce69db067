"""Every launch grid a valid template can ask for fits the device's limits:
at most 65,536 blocks in the second dimension and 2^31 - 1 in the first.
Checked on the host by compiling the grid functions (csrc/tiles.hpp) into a
small program that walks the boundary shapes the ABI allows (widths up to
2^20, heights up to 2^19, at most 2^28 pixels; scan lengths up to 2^31)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_05495_amd", "csrc")

PROGRAM = r"""
#include <algorithm>
#include <cstdio>
#include <vector>
#include "tiles.hpp"
using namespace setrt;
static int bad = 0;
static void check(const char* what, int h, int w, Grid3 g) {
  if (g.x < 1 || g.y < 1 || g.y > 65536u || g.x > 2147483647u || g.z != 1) {
    std::printf("%s %dx%d: grid %u x %u x %u\n", what, h, w, g.x, g.y, g.z);
    ++bad;
  }
}
int main() {
  std::vector<int> widths = {1, 2, 3, 4, 5, 8, 252, 256, 260, 1024, 1028, 2048, 2052, 4096, 6144, 8192,
                             16384, 65536, 1 << 19, (1 << 20) - 4, 1 << 20};
  long long shapes = 0;
  for (int w : widths) {
    const long long hmax = std::min<long long>(1 << 19, (1ll << 28) / w);
    for (long long h : {1ll, 2ll, 3ll, 7ll, 15ll, 16ll, 17ll, hmax / 2 + 1, hmax - 1, hmax}) {
      if (h < 1 || h > hmax) continue;
      ++shapes;
      check("box", (int)h, w, box_grid((int)h, w));
      check("gauss", (int)h, w, gauss_grid((int)h, w));
      check("sobel", (int)h, w, sobel_grid((int)h, w));
      check("hotspot", (int)h, w, hotspot_grid((int)h, w));
      const long long n = h * w;
      if (div9_blocks(n) < 1 || hist_blocks(n) < 1 || div9_blocks(n) > 2147483647u) ++bad;
      if (sobel_partials((int)h, w) < 1) ++bad;
    }
  }
  for (unsigned long long n : {1ull, 2048ull, 2049ull, 1ull << 20, (1ull << 31) - 1, 1ull << 31})
    if (scan_tiles(n) < 1 || scan_tiles(n) > 2147483647u || vec_blocks(n) < 1) ++bad;
  // the row-band choices the stage rooflines were measured for
  struct Case { int h, w, gauss_rows, hot_rows; };
  const Case cases[] = {{1024, 1024, 0, 0}, {2048, 2048, 8, 8}, {1024, 2048, 8, 0}, {1024, 4096, 8, 8},
                        {4096, 4096, 8, 16}, {8192, 8192, 4, 0}, {2048, 2052, 0, 0}, {2048, 6144, 8, 16}};
  for (const Case& c : cases) {
    const int g = gauss_band_path(c.w) ? gauss_band_rows(c.h, c.w) : 0;
    const int t = hotspot_band_rows(c.h, c.w);
    if (g != c.gauss_rows || t != c.hot_rows) {
      std::printf("band rows %dx%d: gauss %d (want %d), thermal %d (want %d)\n", c.h, c.w, g, c.gauss_rows, t,
                  c.hot_rows);
      ++bad;
    }
  }
  std::printf("shapes %lld bad %d\n", shapes, bad);
  return bad ? 1 : 0;
}
"""


def test_every_valid_template_grid_fits_the_launch_limits(tmp_path):
    """Also pins which shapes take the row-band kernels, and with how many rows."""
    src = tmp_path / "grids.cpp"
    exe = tmp_path / "grids"
    src.write_text(PROGRAM)
    r = subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], capture_output=True,
                       text=True)
    if r.returncode != 0:
        pytest.fail("compile failed:\n" + r.stderr[-2000:])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout[-2000:]
    assert "bad 0" in out.stdout
