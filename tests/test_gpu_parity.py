"""GPU parity: every pipeline run through the C ABI on an MI355X against the
CPU oracle on the same seeded inputs.

Bars: integer stages (box sums, quotients, histogram, scan) bit-exact; the
float32 Gaussian within 1e-5 of the convolution of |input| (a relative bound
on the terms summed); Sobel sums within 1e-5 relative; the mask bit-exact
outside the band |mag - 1| <= 1e-5 and the count within that band; vector sums
within max(1e-5 |S|, E) with E the float32 error allowance the oracle returns.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2606_05495_amd import _abi as A
from paper_2606_05495_amd import synth
from paper_2606_05495_amd.runtime import Context, out_header, pinned

pytestmark = pytest.mark.gpu


def _say(*a):
    """Progress and report lines; also appended to the file SET_TEST_REPORT names, if set."""
    print(*a, flush=True)
    sys.stdout.flush()
    path = os.environ.get("SET_TEST_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(" ".join(str(v) for v in a) + "\n")


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _up64(v):
    return (v + 63) // 64 * 64


def _check_header(buf, job_id, tag=None):
    h = out_header(buf)
    assert h["magic"] == A.SET_OUT_MAGIC, hex(int(h["magic"]))
    assert h["canary_ok"] == 1
    assert h["job_id"] == job_id
    if tag is not None:
        assert h["user_tag"] == tag
    return h


# ------------------------------------------------------------------ box / histogram
def _run_images(mode, pipeline, imgs, in_dtype, workers=4, slots=4, flags=A.SET_TF_DEBUG, copy="kernels", **kw):
    h, w = imgs[0].shape
    ctx = Context(mode=mode, workers=workers, slots=slots, **kw)
    tid = ctx.define(pipeline, width=w, height=h, flags=flags, copy=copy)
    ib, ob = ctx.in_bytes(tid), ctx.out_bytes(tid)
    stride = _up64(ob)
    istride = _up64(ib)
    tin, nin = pinned(istride * len(imgs))
    tout, nout = pinned(stride * len(imgs))
    for i, im in enumerate(imgs):
        nin[i * istride:i * istride + ib].view(in_dtype)[:] = im.ravel()
    arr = ctx.job_array(len(imgs))
    arr["host_in"] = tin.data_ptr() + np.arange(len(imgs), dtype=np.uint64) * istride
    arr["in_bytes"] = ib
    arr["host_out"] = tout.data_ptr() + np.arange(len(imgs), dtype=np.uint64) * stride
    arr["out_bytes"] = ob
    arr["user_tag"] = 1000 + np.arange(len(imgs))
    first = ctx.submit_many(tid, arr)
    ctx.drain()
    st = ctx.stats()
    outs = [nout[i * stride:(i + 1) * stride] for i in range(len(imgs))]
    for i in range(len(imgs)):
        _check_header(outs[i], first + i, 1000 + i)
    ctx.close()
    return outs, st


BOX_SHAPES = [(1, 1), (1, 7), (7, 1), (2, 2), (3, 5), (16, 64), (17, 65), (17, 33), (256, 256), (300, 513)]


@pytest.mark.parametrize("mode", ["sync", "set"])
@pytest.mark.parametrize("shape", BOX_SHAPES)
def test_box_hist_parity(torch_gpu, mode, shape):
    _say("box_hist", mode, shape)
    h, w = shape
    rng = np.random.default_rng(h * 1000 + w)
    imgs = [rng.integers(0, 256, shape, dtype=np.uint8), np.full(shape, 255, np.uint8),
            np.zeros(shape, np.uint8), rng.choice(np.array([0, 255], np.uint8), shape)]
    outs, _ = _run_images(mode, "box_hist", imgs, np.uint8)
    s_off = _up64(64 + 1024)
    q_off = _up64(s_off + 2 * h * w)
    for img, o in zip(imgs, outs):
        S, Q, H = oracle.box_hist(img)
        assert np.array_equal(o[64:64 + 1024].view(np.uint32), H)
        assert np.array_equal(o[s_off:s_off + 2 * h * w].view(np.uint16).reshape(h, w), S)
        assert np.array_equal(o[q_off:q_off + h * w].reshape(h, w), Q)


@pytest.mark.parametrize("mode", ["sync", "graph", "batch", "queue", "set"])
def test_box_hist_workload_64_jobs(torch_gpu, mode):
    """64 jobs of 256x256 uint8 (uniform, stream key = seed + job id), 4 streams."""
    _say("box_hist 64 jobs", mode)
    imgs = [synth.box_image(0, j) for j in range(64)]
    outs, st = _run_images(mode, "box_hist", imgs, np.uint8, workers=4, slots=4, flags=0)
    for img, o in zip(imgs, outs):
        assert np.array_equal(o[64:64 + 1024].view(np.uint32), oracle.box_hist(img)[2])
    assert st.completed == 64


# ------------------------------------------------------------------ Gaussian / Sobel
def _check_gauss(img, o, exact_mask=True):
    h, w = img.shape
    ref = oracle.gauss_sobel(img)
    absconv = oracle.gauss_sobel(np.abs(img))["blur"]
    m_off = 128
    b_off = _up64(128 + h * w)
    count = int(o[64:68].view(np.uint32)[0])
    s = float(o[68:72].view(np.float32)[0])
    mask = o[m_off:m_off + h * w].reshape(h, w)
    blur = o[b_off:b_off + 4 * h * w].view(np.float32).reshape(h, w)
    err = np.abs(blur.astype(np.float64) - ref["blur"])
    assert np.all(err <= 1e-5 * absconv + 1e-30), float((err / (absconv + 1e-30)).max())
    outside = np.abs(ref["mag"] - 1.0) > oracle.BAND_EPS
    assert np.array_equal(mask[outside], ref["mask"][outside])
    assert abs(count - ref["count"]) <= ref["band"]
    assert abs(s - ref["sum"]) <= 1e-5 * abs(ref["sum"]) + 1e-6, (s, ref["sum"])
    return ref


# widths that are multiples of 4 take the register-window kernels (ragged
# against the 256-column / 16-row block), the others the LDS-tile kernels
GAUSS_SHAPES = [(1, 1), (1, 9), (9, 1), (2, 3), (5, 5), (16, 64), (17, 65), (33, 17), (100, 130), (256, 256),
                (1, 4), (3, 8), (70, 4), (17, 260), (35, 516), (2, 1028), (257, 264)]


@pytest.mark.parametrize("mode", ["sync", "set"])
@pytest.mark.parametrize("shape", GAUSS_SHAPES)
def test_gauss_sobel_parity(torch_gpu, mode, shape):
    _say("gauss_sobel", mode, shape)
    h, w = shape
    imgs = [synth.normal_image(0, k, h, w) for k in range(3)]
    imgs.append((synth.normal_image(0, 9, h, w) * 4).astype(np.float32))
    outs, _ = _run_images(mode, "gauss_sobel", imgs, np.float32)
    for img, o in zip(imgs, outs):
        _check_gauss(img, o)


@pytest.mark.parametrize("w", [70, 72])
def test_gauss_sobel_pins_on_gpu(torch_gpu, w):
    """Constant image: zero gradient everywhere; impulse: blur = g_i*g_j in float32
    (width 70: LDS-tile kernels, 72: register-window kernels)."""
    _say("gauss_sobel pins", w)
    h = 24
    const = np.full((h, w), 3.25, np.float32)
    imp = np.zeros((h, w), np.float32)
    imp[10, 30] = 1.0
    ramp = (0.25 * np.tile(np.arange(w, dtype=np.float32), (h, 1))).astype(np.float32)
    outs, _ = _run_images("set", "gauss_sobel", [const, imp, ramp], np.float32)
    b_off = _up64(128 + h * w)
    assert int(outs[0][64:68].view(np.uint32)[0]) == 0
    assert float(outs[0][68:72].view(np.float32)[0]) == 0.0
    blur = outs[1][b_off:b_off + 4 * h * w].view(np.float32).reshape(h, w)
    g = oracle.gauss_taps().astype(np.float32)
    for i in range(5):
        for j in range(5):
            assert blur[10 + i - 2, 30 + j - 2] == np.float32(g[i]) * np.float32(g[j])
    mask = outs[2][128:128 + h * w].reshape(h, w)
    assert np.all(mask[:, 3:w - 3] == 1)


@pytest.mark.parametrize("mode", ["sync", "graph", "batch", "queue", "set"])
def test_gauss_sobel_full_size(torch_gpu, mode):
    """1024x1024 N(0,1) images from the 61-image pool, 8 workers x 16 slots."""
    _say("gauss_sobel 1024^2", mode)
    imgs = [synth.normal_image(0, k) for k in range(6)]
    outs, st = _run_images(mode, "gauss_sobel", imgs + imgs, np.float32, workers=8, slots=16, flags=0,
                           callback="host_flag", dispatchers=4)
    for k, img in enumerate(imgs + imgs):
        ref = oracle.gauss_sobel(img, want_images=False)
        o = outs[k]
        count = int(o[64:68].view(np.uint32)[0])
        s = float(o[68:72].view(np.float32)[0])
        assert abs(count - ref["count"]) <= ref["band"]
        assert abs(s - ref["sum"]) <= 1e-5 * abs(ref["sum"])
    # determinism: the same image gives bit-identical results in any slot/stream
    for k in range(6):
        assert np.array_equal(outs[k][64:72], outs[k + 6][64:72])


def test_gauss_sobel_largest_serving_size(torch_gpu):
    """2048x2048, the largest image of the serving mix (16 MiB input), through SET."""
    _say("gauss_sobel 2048^2")
    imgs = [synth.normal_image(3, k, 2048, 2048) for k in range(2)]
    outs, _ = _run_images("set", "gauss_sobel", imgs + imgs[:1], np.float32, workers=2, slots=2, flags=0)
    for k, img in enumerate(imgs + imgs[:1]):
        ref = oracle.gauss_sobel(img, want_images=False)
        assert abs(int(outs[k][64:68].view(np.uint32)[0]) - ref["count"]) <= ref["band"]
        assert abs(float(outs[k][68:72].view(np.float32)[0]) - ref["sum"]) <= 1e-5 * abs(ref["sum"])
    assert np.array_equal(outs[0][64:72], outs[2][64:72])


def test_gauss_sobel_above_2048sq_per_pixel(torch_gpu):
    """2056x2052 (more than 2048^2 pixels: four rows per wave in both stages;
    ragged against the 256-column and 16-row blocks, so lanes past the right
    edge), every pixel of blur and mask."""
    _say("gauss_sobel 2056x2052 per pixel")
    imgs = [synth.normal_image(4, 0, 2056, 2052)]
    outs, _ = _run_images("set", "gauss_sobel", imgs, np.float32, workers=1, slots=1)
    _check_gauss(imgs[0], outs[0])


def test_gauss_sobel_full_width_four_rows_per_pixel(torch_gpu):
    """1210x2048: the width is a multiple of 256 (the full-width window
    kernels, no lane past the right edge) and the image has more than 1024^2
    pixels (four rows per wave in both stages); the height is ragged against
    the 16-row blocks.  Every pixel of blur and mask."""
    _say("gauss_sobel 1210x2048 per pixel")
    imgs = [synth.normal_image(5, 0, 1210, 2048)]
    outs, _ = _run_images("set", "gauss_sobel", imgs, np.float32, workers=1, slots=1)
    _check_gauss(imgs[0], outs[0])


# Widths that are multiples of 2048 take the Gaussian's row-band kernel:
# blocks of 8 waves across 8 rows (4 above 4096^2 pixels), halo columns
# passed between waves in LDS and loaded only at a block's outer edges.
# Heights ragged against the rows of a band; 1, 2, 3 and 4 blocks per band;
# 4097x4096 takes the 4-row bands.
BAND_SHAPES = [(1, 2048), (3, 2048), (6, 4096), (37, 2048), (37, 4096), (9, 6144), (2, 8192), (4097, 4096)]


@pytest.mark.parametrize("shape", BAND_SHAPES)
def test_gauss_sobel_row_bands_per_pixel(torch_gpu, shape):
    _say("gauss_sobel row bands", shape)
    h, w = shape
    imgs = [synth.normal_image(6, k, h, w) for k in range(2)]
    outs, _ = _run_images("set", "gauss_sobel", imgs, np.float32, workers=2, slots=1)
    for img, o in zip(imgs, outs):
        _check_gauss(img, o)


def test_gauss_row_band_impulses_at_wave_and_block_edges(torch_gpu):
    """Impulses on the columns either side of every wave boundary (256k) and
    block boundary (2048) of a 4096-wide image: each blur is exactly the
    float32 product g_i*g_j in its 5x5 neighbourhood and exactly zero
    elsewhere, so a halo pair taken from the wrong wave, block or row shows."""
    _say("gauss row-band impulses")
    h, w = 24, 4096
    cols = [[255, 767, 1279, 2047, 2559, 3071, 3839], [256, 768, 1280, 2048, 2560, 3072, 3840]]
    imgs = []
    for cs in cols:
        im = np.zeros((h, w), np.float32)
        for k, c in enumerate(cs):
            im[4 + 2 * (k % 3) + 4 * (k % 2), c] = 1.0
        imgs.append(im)
    outs, _ = _run_images("set", "gauss_sobel", imgs, np.float32, workers=1, slots=2)
    g = oracle.gauss_taps().astype(np.float32)
    b_off = _up64(128 + h * w)
    for im, o in zip(imgs, outs):
        blur = o[b_off:b_off + 4 * h * w].view(np.float32).reshape(h, w)
        want = np.zeros((h, w), np.float32)
        for y, x in zip(*np.nonzero(im)):
            for i in range(5):
                for j in range(5):
                    want[y + i - 2, x + j - 2] = np.float32(g[i]) * np.float32(g[j])
        assert np.array_equal(blur, want)


# ------------------------------------------------------------------ vector jobs
@pytest.fixture(scope="module")
def vec_pools(torch_gpu):
    L = 1 << 23
    x = synth.vec_pool(0, "x", L)
    y = synth.vec_pool(0, "y", L)
    xd = torch_gpu.from_numpy(x).cuda()
    yd = torch_gpu.from_numpy(y).cuda()
    return x, y, xd, yd


def _run_vec(mode, pools, ns, offs_x, offs_y, avals, workers=4, slots=8, policy=A.SET_SUBMIT_ROUND_ROBIN,
             copy="kernels", **kw):
    x, y, xd, yd = pools
    ctx = Context(mode=mode, workers=workers, slots=slots, submit_policy=policy, **kw)
    tid = ctx.define("saxpy_tanh_sum", max_n=int(max(ns)), x_pool=xd, y_pool=yd, copy=copy)
    k = len(ns)
    tout, nout = pinned(128 * k)
    arr = ctx.job_array(k)
    arr["host_out"] = tout.data_ptr() + np.arange(k, dtype=np.uint64) * 128
    arr["out_bytes"] = 68
    arr["n"] = ns
    arr["a"] = avals
    arr["x_off"] = offs_x
    arr["y_off"] = offs_y
    arr["user_tag"] = np.arange(k)
    first = ctx.submit_many(tid, arr)
    ctx.drain()
    st = ctx.stats()
    res = []
    for i in range(k):
        o = nout[i * 128:(i + 1) * 128]
        _check_header(o, first + i, i)
        res.append(float(o[64:68].view(np.float32)[0]))
    ctx.close()
    return np.array(res), st


@pytest.mark.parametrize("mode", ["sync", "graph", "batch", "queue", "set"])
def test_vector_parity(torch_gpu, vec_pools, mode):
    _say("vector", mode)
    x, y = vec_pools[0], vec_pools[1]
    ns = np.array([1, 2, 3, 4, 5, 1023, 1024, 2047, 2048, 4096, 4097, 65549, 1 << 20, 4194303], np.int64)
    L = len(x)
    rng = np.random.default_rng(5)
    xo = 64 * (rng.integers(0, (L - ns) // 64))
    yo = 64 * (rng.integers(0, (L - ns) // 64))
    xo[3] += 1  # misaligned windows take the scalar path
    yo[5] += 3
    av = rng.uniform(0.5, 2, len(ns)).astype(np.float32)
    got, _ = _run_vec(mode, vec_pools, ns, xo, yo, av)
    by_floor = 0
    for i, n in enumerate(ns):
        S, E = oracle.saxpy_tanh_sum(x[xo[i]:xo[i] + n], y[yo[i]:yo[i] + n], av[i])
        ok, fl = oracle.vec_verdict(got[i], S, E)
        assert ok, (n, got[i], S, E)
        by_floor += fl
    _say("vector", mode, "passed only by the floor E: %d of %d" % (by_floor, len(ns)))


def test_vector_batch_graph_spans_slots(torch_gpu, vec_pools):
    """Batch-sync graphs of 10 chains on 3 workers x 4 slots (chain i in slot
    i // 3 of worker i % 3), 25 jobs: 2 full batches and one of 5 at drain;
    every header (magic, canaries, job id, tag) and every result against the
    oracle."""
    _say("vector batch graph of 10 chains on 3 workers x 4 slots")
    x, y = vec_pools[0], vec_pools[1]
    rng = np.random.default_rng(11)
    ns = rng.integers(1, 300000, 25).astype(np.int64)
    L = len(x)
    xo = 64 * (rng.integers(0, (L - ns) // 64))
    yo = 64 * (rng.integers(0, (L - ns) // 64))
    av = rng.uniform(0.5, 2, len(ns)).astype(np.float32)
    got, st = _run_vec("batch", vec_pools, ns, xo, yo, av, workers=3, slots=4, batch_size=10)
    assert st.batches == 3
    for i, n in enumerate(ns):
        S, E = oracle.saxpy_tanh_sum(x[xo[i]:xo[i] + n], y[yo[i]:yo[i] + n], av[i])
        assert abs(got[i] - S) <= oracle.vec_tolerance(S, E), (n, got[i], S, E)


def test_vector_pins_on_gpu(torch_gpu):
    """a=16, x=1, y=0 saturates tanh to exactly 1.0f, so S = n exactly; x=y=0 gives 0."""
    _say("vector pins")
    import torch
    L = 1 << 22
    ones = torch.ones(L, dtype=torch.float32, device="cuda")
    zeros = torch.zeros(L, dtype=torch.float32, device="cuda")
    ns = np.array([1, 4096, 4097, 1 << 20, 4194303], np.int64)
    got, _ = _run_vec("set", (None, None, ones, zeros), ns, np.zeros(5, np.int64), np.zeros(5, np.int64),
                      np.full(5, 16.0, np.float32))
    assert np.array_equal(got, ns.astype(np.float32))
    got0, _ = _run_vec("set", (None, None, zeros, zeros), ns, np.zeros(5, np.int64), np.zeros(5, np.int64),
                       np.full(5, 1.5, np.float32))
    assert np.all(got0 == 0.0)


@pytest.fixture(scope="module")
def ternary_pools(torch_gpu):
    """x in {-1, 0, 1} (seeded), y = 0: with a = 16 every tanh(a*x + y) is
    exactly -1, 0 or 1 in float32 (tanh(16) = 1 - 2.5e-14 rounds to 1), so a
    job's S is an integer of magnitude < 2^24 and every partial sum of it is
    exact in any order: S equals the integer sum of its x window."""
    L = 1 << 23
    x = np.random.default_rng(21).integers(-1, 2, L).astype(np.float32)
    y = np.zeros(L, np.float32)
    return x, y, torch_gpu.from_numpy(x).cuda(), torch_gpu.from_numpy(y).cuda()


# n spans one item / block up to the largest job, with ragged tails
EXACT_NS = np.array([1, 3, 4095, 4097, 65549, (1 << 20) + 3, 4194303], np.int64)


def _misaligned_windows(ns, L, seed):
    """Window offsets cycling through every alignment mod 4 for x and y."""
    rng = np.random.default_rng(seed)
    xo = 64 * rng.integers(0, (L - ns - 4) // 64) + np.arange(len(ns)) % 4
    yo = 64 * rng.integers(0, (L - ns - 4) // 64) + (np.arange(len(ns)) * 3 + 1) % 4
    return xo.astype(np.int64), yo.astype(np.int64)


@pytest.mark.parametrize("mode", ["sync", "graph", "batch", "queue", "set"])
def test_vector_exact_sums_misaligned(torch_gpu, ternary_pools, mode):
    """Per-job path: S equals the exact integer sum of the x window for every
    alignment of the x and y windows (16-byte path and scalar path), so one
    element dropped or counted twice anywhere (tile tails included) fails."""
    _say("vector exact sums, misaligned windows", mode)
    x = ternary_pools[0]
    ns = np.concatenate([EXACT_NS, EXACT_NS[3:]])
    xo, yo = _misaligned_windows(ns, len(x), 31)
    xo[len(EXACT_NS):] -= xo[len(EXACT_NS):] % 4  # the second copy: 4-aligned x windows
    yo[len(EXACT_NS):] -= yo[len(EXACT_NS):] % 4
    got, _ = _run_vec(mode, ternary_pools, ns, xo, yo, np.full(len(ns), 16.0, np.float32))
    for i, n in enumerate(ns):
        exact = int(np.sum(x[xo[i]:xo[i] + n].astype(np.int64)))
        S, _ = oracle.saxpy_tanh_sum(x[xo[i]:xo[i] + n], ternary_pools[1][yo[i]:yo[i] + n], 16.0)
        # the float64 oracle carries tanh(16)'s residue 2.5e-14 per nonzero
        # element; float32 rounds it away
        assert abs(S - exact) <= n * 2.6e-14 and np.float32(S) == np.float32(exact)
        assert got[i] == np.float32(exact), (mode, int(n), int(xo[i]) % 4, int(yo[i]) % 4, got[i], exact)


@pytest.mark.parametrize("tile,block", [(1024, 0), (4096, 0), (65536, 0), (4096, 128), (1024, 512), (65536, 1024)])
def test_vector_batching_exact_sums_misaligned(torch_gpu, ternary_pools, tile, block):
    """Batched path (persistent kernel over a descriptor table): the same
    exact sums for every window alignment, work-item size and block size of
    the work-item kernel."""
    _say("vector batching exact sums, tile", tile, "block", block)
    x, y, xd, yd = ternary_pools
    ns = np.concatenate([EXACT_NS, EXACT_NS])
    xo, yo = _misaligned_windows(ns, len(x), 37)
    xo[len(EXACT_NS):] -= xo[len(EXACT_NS):] % 4
    yo[len(EXACT_NS):] -= yo[len(EXACT_NS):] % 4
    jobs = np.zeros(len(ns), dtype=A.VEC_JOB_DTYPE)
    jobs["n"], jobs["a"], jobs["x_off"], jobs["y_off"] = ns, 16.0, xo, yo
    tune = A.set_vec_tuning()
    for b in range(64):
        tune.tile_elems[b] = tile
    ctx = Context(mode="set", workers=2, slots=4)
    tid = ctx.define("saxpy_batch", max_n=1 << 22, x_pool=xd, y_pool=yd, batch_max=8, tiles_max=8192, block=block)
    res, _ = ctx.run_vector_jobs(tid, jobs, tuning=tune)
    ctx.close()
    for i, n in enumerate(ns):
        exact = int(np.sum(x[xo[i]:xo[i] + n].astype(np.int64)))
        assert res[i] == np.float32(exact), (tile, int(n), int(xo[i]) % 4, int(yo[i]) % 4, res[i], exact)


def test_vector_workload_sample(torch_gpu, vec_pools):
    """A sample of the uneven vector workload (n log-uniform in [4096, 4194304)), with stealing."""
    _say("vector workload sample")
    x, y = vec_pools[0], vec_pools[1]
    jobs = synth.vec_jobs(0, 120, pool_len=len(x))
    got, st = _run_vec("set", vec_pools, jobs["n"], jobs["x_off"], jobs["y_off"], jobs["a"], workers=8, slots=16,
                       policy=A.SET_SUBMIT_SKEW0, callback="host_flag", dispatchers=4)
    assert st.stolen > 0
    by_floor = 0
    for i in range(len(got)):
        n = int(jobs["n"][i])
        S, E = oracle.saxpy_tanh_sum(x[jobs["x_off"][i]:jobs["x_off"][i] + n],
                                     y[jobs["y_off"][i]:jobs["y_off"][i] + n], jobs["a"][i])
        ok, fl = oracle.vec_verdict(got[i], S, E)
        assert ok, (i, n, got[i], S, E)
        by_floor += fl
    _say("vector workload sample: passed only by the floor E: %d of %d" % (by_floor, len(got)))
    # alone vs in the mix: bit-identical
    alone, _ = _run_vec("sync", vec_pools, jobs["n"][:10], jobs["x_off"][:10], jobs["y_off"][:10], jobs["a"][:10],
                        workers=1, slots=1)
    assert np.array_equal(alone, got[:10])


# ------------------------------------------------------------------ scan
def _run_scan_flags(mode, inputs, max_n, flags, copy):
    return _run_scan(mode, inputs, max_n, copy=copy, extra_flags=flags)


def _run_scan(mode, inputs, max_n, low32=False, workers=4, slots=4, copy="kernels", extra_flags=0, pipeline="scan",
              **kw):
    ctx = Context(mode=mode, workers=workers, slots=slots, **kw)
    tid = ctx.define(pipeline, max_n=max_n, flags=(A.SET_TF_SCAN_LOW32 if low32 else 0) | extra_flags, copy=copy)
    k = len(inputs)
    ib = [4 * len(v) for v in inputs]
    ob = [ctx.out_bytes(tid, len(v)) for v in inputs]
    tin, nin = pinned(sum(_up64(v) for v in ib))
    tout, nout = pinned(sum(_up64(v) for v in ob))
    arr = ctx.job_array(k)
    oi = oo = 0
    offs = []
    for i, v in enumerate(inputs):
        nin[oi:oi + ib[i]].view(np.int32)[:] = v
        arr[i]["host_in"] = tin.data_ptr() + oi
        arr[i]["in_bytes"] = ib[i]
        arr[i]["host_out"] = tout.data_ptr() + oo
        arr[i]["out_bytes"] = ob[i]
        arr[i]["n"] = len(v)
        offs.append(oo)
        oi += _up64(ib[i])
        oo += _up64(ob[i])
    first = ctx.submit_many(tid, arr)
    ctx.drain()
    res = []
    for i, v in enumerate(inputs):
        o = nout[offs[i]:offs[i] + ob[i]]
        _check_header(o, first + i)
        res.append(o[64:].view(np.uint32 if low32 else np.int64).copy())
    ctx.close()
    return res


@pytest.mark.parametrize("mode", ["sync", "graph", "batch", "queue", "set"])
def test_scan_parity(torch_gpu, mode):
    _say("scan", mode)
    rng = np.random.default_rng(3)
    ns = [1, 7, 8, 2047, 2048, 2049, 4096, 100003, 1 << 18]
    inputs = [rng.integers(-(1 << 20), (1 << 20) + 1, n).astype(np.int32) for n in ns]
    inputs.append(np.full(50000, np.iinfo(np.int32).max, np.int32))
    inputs.append(np.full(50000, np.iinfo(np.int32).min, np.int32))
    res = _run_scan(mode, inputs, max_n=1 << 18)
    for v, r in zip(inputs, res):
        assert np.array_equal(r, oracle.scan(v))


def test_scan_full_size_and_low32(torch_gpu):
    """2^21 int32 inputs in [-2^20, 2^20]; the int64 sums reach 2^41."""
    _say("scan 2^21")
    inputs = [synth.scan_input(0, k) for k in range(3)] + [np.full(1 << 21, 1 << 20, np.int32)]
    res = _run_scan("set", inputs, max_n=1 << 21, workers=8, slots=4)
    for v, r in zip(inputs, res):
        assert np.array_equal(r, oracle.scan(v))
    assert res[-1][-1] == 1 << 41
    res32 = _run_scan("set", inputs[:2], max_n=1 << 21, low32=True)
    for v, r in zip(inputs[:2], res32):
        assert np.array_equal(r, (oracle.scan(v) & 0xFFFFFFFF).astype(np.uint32))


# ------------------------------------------------------------------ scheduling on the device
@pytest.mark.parametrize("callback,nd,ncb,sp", [("event_chain", 1, 0, 0), ("event_chain", 3, 0, 0),
                                                ("event_chain", 3, 2, 0), ("event_chain", 1, 4, 0),
                                                ("same_stream", 1, 0, 0), ("event_poll", 1, 0, 0),
                                                ("host_flag", 1, 0, 0), ("event_poll", 4, 0, 0),
                                                ("host_flag", 3, 0, 0), ("event_blocking", 1, 0, 0),
                                                ("event_blocking", 4, 0, 0), ("event_poll", 4, 0, 1),
                                                ("host_flag", 1, 0, 1)])
def test_set_mode_callbacks_and_steals(torch_gpu, callback, nd, ncb, sp):
    """Skewed submission on the GPU: steals retarget jobs to thieves' slots; results stay exact
    (one dispatcher thread, or several each owning a share of the workers; event chaining on
    one callback stream shared by the workers, on two, or on one per worker; victims taken as
    printed, or only busy ones)."""
    _say("set callbacks", callback, nd, ncb, sp)
    imgs = [synth.box_image(0, j) for j in range(96)]
    ctx = Context(mode="set", workers=4, slots=4, callback=callback, submit_policy=A.SET_SUBMIT_SKEW0,
                  dispatchers=nd, callback_streams=ncb, steal_policy=sp)
    tid = ctx.define("box_hist", width=256, height=256)
    ib, ob = ctx.in_bytes(tid), ctx.out_bytes(tid)
    tin, nin = pinned(ib * 96)
    tout, nout = pinned(_up64(ob) * 96)
    nin[:] = np.concatenate([im.ravel() for im in imgs])
    arr = ctx.job_array(96)
    arr["host_in"] = tin.data_ptr() + np.arange(96, dtype=np.uint64) * ib
    arr["in_bytes"] = ib
    arr["host_out"] = tout.data_ptr() + np.arange(96, dtype=np.uint64) * _up64(ob)
    arr["out_bytes"] = ob
    ctx.submit_many(tid, arr)
    ctx.drain()
    st = ctx.stats()
    times = {int(r["job_id"]): r for r in ctx.job_times()}
    ctx.close()
    for j in range(96):
        o = nout[j * _up64(ob):(j + 1) * _up64(ob)]
        h = _check_header(o, j)
        assert h["worker"] == times[j]["worker"] and h["slot"] == times[j]["slot"]
        assert np.array_equal(o[64:64 + 1024].view(np.uint32), oracle.box_hist(imgs[j])[2])
    assert st.completed == 96
    # As printed, skewed submission must produce steals.  Under SET_STEAL_BUSY
    # a victim that keeps up (its permit back before a thief looks) is never
    # robbed, so steals there depend on timing; the fake-backend tests pin them.
    if sp == A.SET_STEAL_ANY:
        assert st.stolen > 0


# ------------------------------------------------------------------ graph memcpy nodes instead of copy kernels
@pytest.mark.parametrize("mode", ["sync", "graph", "batch", "set"])
def test_memcpy_nodes_all_pipelines(torch_gpu, vec_pools, mode):
    """The same chains with the H2D/D2H as graph memcpy nodes (hipMemcpyAsync in the synchronous model)."""
    _say("memcpy nodes", mode)
    imgs8 = [synth.box_image(0, j, 37, 201) for j in range(5)]
    outs, _ = _run_images(mode, "box_hist", imgs8, np.uint8, copy="nodes")
    s_off = _up64(64 + 1024)
    q_off = _up64(s_off + 2 * 37 * 201)
    for img, o in zip(imgs8, outs):
        S, Q, H = oracle.box_hist(img)
        assert np.array_equal(o[64:64 + 1024].view(np.uint32), H)
        assert np.array_equal(o[q_off:q_off + 37 * 201].reshape(37, 201), Q)
    imgsf = [synth.normal_image(0, k, 70, 99) for k in range(5)]
    outs, _ = _run_images(mode, "gauss_sobel", imgsf, np.float32, copy="nodes")
    for img, o in zip(imgsf, outs):
        _check_gauss(img, o)
    big = [synth.normal_image(0, k) for k in range(3)]
    outs, _ = _run_images(mode, "gauss_sobel", big, np.float32, workers=8, slots=4, flags=0, copy="nodes")
    for img, o in zip(big, outs):
        ref = oracle.gauss_sobel(img, want_images=False)
        assert abs(int(o[64:68].view(np.uint32)[0]) - ref["count"]) <= ref["band"]
        assert abs(float(o[68:72].view(np.float32)[0]) - ref["sum"]) <= 1e-5 * abs(ref["sum"])
    rng = np.random.default_rng(11)
    ins = [rng.integers(-(1 << 20), (1 << 20) + 1, n).astype(np.int32) for n in (1, 5, 4097, 1 << 21)]
    for v, r in zip(ins, _run_scan(mode, ins, max_n=1 << 21, copy="nodes")):
        assert np.array_equal(r, oracle.scan(v))
    x, y = vec_pools[0], vec_pools[1]
    ns = np.array([3, 4096, 70001], np.int64)
    got, _ = _run_vec(mode, vec_pools, ns, np.array([0, 64, 128]), np.array([64, 0, 4]),
                      np.full(3, 1.25, np.float32), copy="nodes")
    for i, n in enumerate(ns):
        xo, yo = [0, 64, 128][i], [64, 0, 4][i]
        S, E = oracle.saxpy_tanh_sum(x[xo:xo + n], y[yo:yo + n], 1.25)
        assert abs(got[i] - S) <= oracle.vec_tolerance(S, E)


# ------------------------------------------------------------------ bucketed persistent batching
@pytest.mark.parametrize("mode,copy", [("set", "nodes"), ("set", "kernels"), ("sync", "kernels"), ("batch", "nodes")])
def test_vector_batching_parity(torch_gpu, vec_pools, mode, copy):
    """Uneven vector jobs through size-bucketed persistent batches: each result matches the oracle,
    and re-batching the same jobs in another order gives bit-identical results (a job's reduction
    order depends only on its length and its bucket's work-item size)."""
    _say("vector batching", mode, copy)
    x, y, xd, yd = vec_pools
    js = synth.vec_jobs(2, 200, pool_len=len(x))
    jobs = np.zeros(200, dtype=A.VEC_JOB_DTYPE)
    for f in ("n", "a", "x_off", "y_off"):
        jobs[f] = js[f]
    jobs["x_off"][:5] += 1  # misaligned windows take the scalar path
    ctx = Context(mode=mode, workers=4, slots=4)
    tid = ctx.define("saxpy_batch", max_n=1 << 22, x_pool=xd, y_pool=yd, batch_max=32, tiles_max=1024, copy=copy)
    res, nb = ctx.run_vector_jobs(tid, jobs)
    assert nb >= 10
    by_floor = 0
    for i in range(200):
        n = int(jobs["n"][i])
        xo, yo = int(jobs["x_off"][i]), int(jobs["y_off"][i])
        S, E = oracle.saxpy_tanh_sum(x[xo:xo + n], y[yo:yo + n], jobs["a"][i])
        ok, fl = oracle.vec_verdict(res[i], S, E)
        assert ok, (i, n, res[i], S, E)
        by_floor += fl
    _say("vector batching", mode, copy, "passed only by the floor E: %d of 200" % by_floor)
    perm = np.random.default_rng(9).permutation(200)
    res2, _ = ctx.run_vector_jobs(tid, jobs[perm])
    assert np.array_equal(res2, res[perm])
    st = ctx.stats()
    assert st.failed == 0
    ctx.close()


@pytest.mark.parametrize("block", [128, 512, 1024])
def test_vector_batching_block_sizes(torch_gpu, vec_pools, block):
    """The work-item kernel at each block size: every job within the oracle's
    tolerance, bit-identical when re-batched in another order (the block is
    fixed per template), and a bad block size refused."""
    _say("vector batching block", block)
    x, y, xd, yd = vec_pools
    js = synth.vec_jobs(6, 120, pool_len=len(x))
    jobs = np.zeros(120, dtype=A.VEC_JOB_DTYPE)
    for f in ("n", "a", "x_off", "y_off"):
        jobs[f] = js[f]
    jobs["y_off"][:4] += 3
    ctx = Context(mode="set", workers=4, slots=4)
    tid = ctx.define("saxpy_batch", max_n=1 << 22, x_pool=xd, y_pool=yd, batch_max=16, tiles_max=1024, block=block)
    res, _ = ctx.run_vector_jobs(tid, jobs)
    for i in range(120):
        n, xo, yo = int(jobs["n"][i]), int(jobs["x_off"][i]), int(jobs["y_off"][i])
        S, E = oracle.saxpy_tanh_sum(x[xo:xo + n], y[yo:yo + n], jobs["a"][i])
        assert abs(float(res[i]) - S) <= oracle.vec_tolerance(S, E), (block, i, n, res[i], S)
    perm = np.random.default_rng(3).permutation(120)
    res2, _ = ctx.run_vector_jobs(tid, jobs[perm])
    assert np.array_equal(res2.view(np.uint32), res[perm].view(np.uint32))
    with pytest.raises(A.SetError):
        ctx.define("saxpy_batch", max_n=1 << 22, x_pool=xd, y_pool=yd, batch_max=16, tiles_max=1024, block=96)
    ctx.close()


def test_device_copy_reference(torch_gpu):
    """The bandwidth reference of the stage tables: a cold copy of 8 MiB takes a
    plausible time (within 1 to 1000 us, and no faster than 8 TB/s allows)."""
    _say("device copy reference")
    ctx = Context(mode="set", workers=2, slots=2)
    us = ctx.time_device_copy(8 << 20, 50)
    assert 8 * 2 ** 20 / (us * 1e-6) <= 8.0e12 and 1.0 <= us <= 1000.0, us
    ctx.close()


@pytest.mark.parametrize("mode", ["set", "sync", "batch", "queue"])
def test_empty_inputs_on_gpu(torch_gpu, vec_pools, mode):
    """Empty submissions and empty vector batches launch nothing and count
    nothing on the HIP backend; the context then runs real jobs normally."""
    _say("empty inputs", mode)
    x, y, xd, yd = vec_pools
    ctx = Context(mode=mode, workers=2, slots=2)
    tid = ctx.define("saxpy_tanh_sum", max_n=1 << 16, x_pool=xd, y_pool=yd)
    tb = ctx.define("saxpy_batch", max_n=1 << 16, x_pool=xd, y_pool=yd, batch_max=4, tiles_max=64)
    ctx.submit_many(tid, ctx.job_array(0))
    ctx.drain(timeout_ns=int(5e9))
    res, nb = ctx.run_vector_jobs(tb, np.zeros(0, dtype=A.VEC_JOB_DTYPE))
    assert nb == 0 and res.size == 0
    assert ctx.stats().submitted == 0
    tout, nout = pinned(128)
    ctx.submit(tid, host_out=tout.data_ptr(), out_bytes=68, n=77, a=1.5, x_off=64, y_off=128)
    ctx.drain()
    S, E = oracle.saxpy_tanh_sum(x[64:64 + 77], y[128:128 + 77], 1.5)
    assert abs(float(nout[64:68].view(np.float32)[0]) - S) <= oracle.vec_tolerance(S, E)
    ctx.close()
    A.set_run_vector_jobs_noalloc(0, 0, xd.data_ptr(), yd.data_ptr(), len(x), 1 << 16, 0, 0, 0)  # count 0: nothing


def test_vector_batching_pins(torch_gpu):
    """Saturated tanh gives S = n exactly through the batched path too."""
    _say("vector batching pins")
    import torch
    L = 1 << 22
    ones = torch.ones(L, dtype=torch.float32, device="cuda")
    zeros = torch.zeros(L, dtype=torch.float32, device="cuda")
    ns = np.array([1, 3, 4096, 4097, 65536, 1 << 20, 4194303, 4194304], np.int64)
    jobs = np.zeros(len(ns), dtype=A.VEC_JOB_DTYPE)
    jobs["n"] = ns
    jobs["a"] = 16.0
    ctx = Context(mode="set", workers=2, slots=4)
    tid = ctx.define("saxpy_batch", max_n=1 << 22, x_pool=ones, y_pool=zeros, batch_max=4, tiles_max=4096)
    res, _ = ctx.run_vector_jobs(tid, jobs)
    assert np.array_equal(res, ns.astype(np.float32))
    ctx.close()


# ------------------------------------------------------------------ serving: alone vs in the mix
def test_serve_alone_vs_mix(torch_gpu, vec_pools):
    """Requests arriving while others run are admitted as slots and memory free up; every result
    equals the same request run alone, bit for bit, and matches the oracle."""
    _say("serve alone vs mix")
    x, y, xd, yd = vec_pools
    sides = (64, 128, 256)
    ctx = Context(mode="set", workers=8, slots=4, mem_budget=256 << 20, callback="event_poll")
    timg = {s: ctx.define("gauss_sobel", width=s, height=s, copy="kernels") for s in sides}
    tvec = ctx.define("saxpy_batch", max_n=1 << 20, x_pool=xd, y_pool=yd, batch_max=64, tiles_max=4096, copy="kernels")
    pools = {s: [synth.normal_image(4, k, s, s) for k in range(5)] for s in sides}
    n_req = 240
    arr = synth.poisson_arrivals(7, 4000.0, 1.0)[:n_req]
    mix = synth.serve_mix(7, n_req)
    vj = synth.vec_jobs(7, n_req, pool_len=len(x), n_span=256.0)
    req = np.zeros(n_req, dtype=A.REQUEST_DTYPE)
    req["t_arrival_ns"] = (arr * 1e9).astype(np.uint64)
    req["worker_hint"] = -1
    tin, nin = pinned(n_req * 4 * 256 * 256)
    tout, nout = pinned(n_req * 128)
    for i in range(n_req):
        if mix["kind"][i] == 0:
            s = sides[mix["side_idx"][i] % 3]
            img = pools[s][mix["pool_idx"][i] % 5]
            off = i * 4 * 256 * 256
            nin[off:off + 4 * s * s].view(np.float32)[:] = img.ravel()
            req[i]["template_id"] = timg[s]
            req[i]["host_in"] = tin.data_ptr() + off
            req[i]["in_bytes"] = 4 * s * s
            req[i]["host_out"] = tout.data_ptr() + 128 * i
            req[i]["out_bytes"] = 72
        else:
            req[i]["template_id"] = tvec
            req[i]["n"] = vj["n"][i]
            req[i]["a"] = vj["a"][i]
            req[i]["x_off"] = vj["x_off"][i]
            req[i]["y_off"] = vj["y_off"][i]
    vres = np.zeros(n_req, np.float32)
    done, st = A.set_serve(ctx.h, req, None, vres)
    assert st.completed == n_req and st.failed == 0, (st.completed, st.failed)
    assert np.all(done >= req["t_arrival_ns"])
    assert st.vec_batches < int(np.sum(mix["kind"] == 1))  # vector requests shared batches
    assert ctx.stats().mem_high_water <= 256 << 20
    mixed_img = nout.reshape(n_req, 128)[:, 64:72].copy()
    # alone: one request at a time through the same templates
    alone_vec = np.zeros(n_req, np.float32)
    for i in range(n_req):
        if mix["kind"][i] == 0:
            s = sides[mix["side_idx"][i] % 3]
            r = ctx.submit(timg[s], host_in=int(req[i]["host_in"]), in_bytes=4 * s * s,
                           host_out=tout.data_ptr() + 128 * i, out_bytes=72)
            ctx.drain()
            img = pools[s][mix["pool_idx"][i] % 5]
            ref = oracle.gauss_sobel(img, want_images=False)
            o = nout[128 * i:128 * i + 128]
            assert abs(int(o[64:68].view(np.uint32)[0]) - ref["count"]) <= ref["band"]
            assert abs(float(o[68:72].view(np.float32)[0]) - ref["sum"]) <= 1e-5 * abs(ref["sum"])
        else:
            one = np.zeros(1, dtype=A.VEC_JOB_DTYPE)
            for f in ("n", "a", "x_off", "y_off"):
                one[f] = req[i][f]
            res, _ = ctx.run_vector_jobs(tvec, one)
            alone_vec[i] = res[0]
            n, xo, yo = int(req[i]["n"]), int(req[i]["x_off"]), int(req[i]["y_off"])
            S, E = oracle.saxpy_tanh_sum(x[xo:xo + n], y[yo:yo + n], req[i]["a"])
            assert abs(res[0] - S) <= oracle.vec_tolerance(S, E)
    alone_img = nout.reshape(n_req, 128)[:, 64:72].copy()
    vec = mix["kind"] == 1
    assert np.array_equal(alone_vec[vec], vres[vec])
    assert np.array_equal(alone_img[~vec], mixed_img[~vec])
    ctx.close()


@pytest.mark.parametrize("callback,inflight,dispatchers,vec_copy",
                         [("event_poll", 0, 1, "kernels"), ("host_flag", 1, 4, "async_in")])
def test_serve_alone_vs_mix_full_sizes(torch_gpu, vec_pools, callback, inflight, dispatchers, vec_copy):
    """The serving mix at its own image sizes (256^2, 512^2, 1024^2, 2048^2 beside vector jobs) under a
    device-memory budget that binds: at most a few 2048^2 slots fit at once, so later arrivals wait for
    memory, and admission must still never exceed the budget.  Each image request gives the same bits
    alone as in the mix and matches the oracle; each vector request likewise.  Second case: the serving
    benchmark's settings (completion words, one job in flight per worker, 4 dispatcher threads, DMA
    input copies for the vector batches' tables too)."""
    _say("serve alone vs mix, full sizes", callback, inflight, dispatchers, vec_copy)
    x, y, xd, yd = vec_pools
    sides = synth.SERVE_SIDES
    budget = 96 << 20
    ctx = Context(mode="set", workers=8, slots=4, mem_budget=budget, callback=callback, inflight=inflight,
                  dispatchers=dispatchers)
    timg = {s: ctx.define("gauss_sobel", width=s, height=s, copy="async_in") for s in sides}
    tvec = ctx.define("saxpy_batch", max_n=1 << 20, x_pool=xd, y_pool=yd, batch_max=64, tiles_max=4096, copy=vec_copy)
    fp = {s: A.set_template_footprint(ctx.cfg, ctx.templates[timg[s]])[0] for s in sides}
    assert 2 * fp[2048] < budget < 4 * fp[2048]
    P = 3
    pools = {s: list(synth.serve_image_pool(0, s, count=P)) for s in sides}
    refs = {(s, k): oracle.gauss_sobel(pools[s][k], want_images=False) for s in sides for k in range(P)}
    offs, total = {}, 0
    for s in sides:
        offs[s] = total
        total += P * 4 * s * s
    tin, nin = pinned(total)
    for s in sides:
        for k in range(P):
            nin[offs[s] + k * 4 * s * s:offs[s] + (k + 1) * 4 * s * s].view(np.float32)[:] = pools[s][k].ravel()
    n_req = 160
    arr = synth.poisson_arrivals(9, 20000.0, 1.0)[:n_req]
    mix = synth.serve_mix(9, n_req)
    vj = synth.vec_jobs(9, n_req, pool_len=len(x), n_span=256.0)
    req = np.zeros(n_req, dtype=A.REQUEST_DTYPE)
    req["t_arrival_ns"] = (arr * 1e9).astype(np.uint64)
    req["worker_hint"] = -1
    tout, nout = pinned(n_req * 128)
    img = mix["kind"] == 0
    side = np.array(sides)[mix["side_idx"]]
    pk = mix["pool_idx"] % P
    for i in range(n_req):
        if img[i]:
            s = int(side[i])
            req[i]["template_id"] = timg[s]
            req[i]["host_in"] = tin.data_ptr() + offs[s] + int(pk[i]) * 4 * s * s
            req[i]["in_bytes"] = 4 * s * s
            req[i]["host_out"] = tout.data_ptr() + 128 * i
            req[i]["out_bytes"] = 72
        else:
            req[i]["template_id"] = tvec
            for f in ("n", "a", "x_off", "y_off"):
                req[i][f] = vj[f][i]
    assert np.sum(img & (side == 2048)) >= 8
    vres = np.zeros(n_req, np.float32)
    done, st = A.set_serve(ctx.h, req, None, vres)
    assert st.completed == n_req and st.failed == 0, (st.completed, st.failed)
    assert np.all(done >= req["t_arrival_ns"])
    hw = ctx.stats().mem_high_water
    _say("serve full sizes: memory high water %d of %d, max backlog %d" % (hw, budget, st.max_backlog))
    assert budget // 2 <= hw <= budget  # the budget was approached and held
    mixed = nout.reshape(n_req, 128)[:, 64:72].copy()
    for i in np.flatnonzero(img):
        s = int(side[i])
        r = refs[(s, int(pk[i]))]
        o = mixed[i]
        assert abs(int(o[0:4].view(np.uint32)[0]) - r["count"]) <= r["band"], (i, s)
        assert abs(float(o[4:8].view(np.float32)[0]) - r["sum"]) <= 1e-5 * abs(r["sum"]), (i, s)
    # alone: each request by itself through the same templates
    nout[:] = 0
    for i in range(n_req):
        if img[i]:
            s = int(side[i])
            ctx.submit(timg[s], host_in=int(req[i]["host_in"]), in_bytes=4 * s * s, host_out=tout.data_ptr() + 128 * i,
                       out_bytes=72)
            ctx.drain()
        else:
            one = np.zeros(1, dtype=A.VEC_JOB_DTYPE)
            for f in ("n", "a", "x_off", "y_off"):
                one[f] = req[i][f]
            res, _ = ctx.run_vector_jobs(tvec, one)
            assert res[0].view(np.uint32) == vres[i].view(np.uint32), i
            n, xo, yo = int(req[i]["n"]), int(req[i]["x_off"]), int(req[i]["y_off"])
            S, E = oracle.saxpy_tanh_sum(x[xo:xo + n], y[yo:yo + n], req[i]["a"])
            assert abs(res[0] - S) <= oracle.vec_tolerance(S, E)
    alone = nout.reshape(n_req, 128)[:, 64:72].copy()
    assert np.array_equal(alone[img], mixed[img])
    ctx.close()


# ------------------------------------------------------------------ stream-captured templates
@pytest.mark.parametrize("mode,copy", [("set", "kernels"), ("set", "nodes"), ("graph", "kernels")])
def test_captured_templates_match_explicit(torch_gpu, vec_pools, mode, copy):
    """Graphs built by stream capture of the launch sequence give bit-identical results to
    explicitly built graphs, for every pipeline, with per-job rebinding working on captured nodes."""
    _say("captured templates", mode, copy)
    imgs = [synth.normal_image(0, k, 96, 130) for k in range(6)]
    a, _ = _run_images(mode, "gauss_sobel", imgs, np.float32, copy=copy)
    b, _ = _run_images(mode, "gauss_sobel", imgs, np.float32, copy=copy, flags=A.SET_TF_DEBUG | A.SET_TF_CAPTURE)
    for x, y in zip(a, b):
        assert np.array_equal(x[64:], y[64:])
    imgs8 = [synth.box_image(0, j, 64, 200) for j in range(6)]
    a, _ = _run_images(mode, "box_hist", imgs8, np.uint8, copy=copy, flags=0)
    b, _ = _run_images(mode, "box_hist", imgs8, np.uint8, copy=copy, flags=A.SET_TF_CAPTURE)
    for x, y, im in zip(a, b, imgs8):
        assert np.array_equal(x[64:64 + 1024], y[64:64 + 1024])
        assert np.array_equal(y[64:64 + 1024].view(np.uint32), oracle.box_hist(im)[2])
    rng = np.random.default_rng(2)
    ins = [rng.integers(-(1 << 20), (1 << 20) + 1, n).astype(np.int32) for n in (7, 4097, 1 << 20)]
    for v, r in zip(ins, _run_scan_flags(mode, ins, 1 << 20, A.SET_TF_CAPTURE, copy)):
        assert np.array_equal(r, oracle.scan(v))
    x, y, xd, yd = vec_pools
    ctx = Context(mode=mode, workers=2, slots=4)
    tv = ctx.define("saxpy_tanh_sum", max_n=1 << 20, x_pool=xd, y_pool=yd, flags=A.SET_TF_CAPTURE, copy=copy)
    tout, nout = pinned(128 * 3)
    ns = [5, 4096, 1 << 20]
    for i, n in enumerate(ns):
        ctx.submit(tv, host_out=tout.data_ptr() + 128 * i, out_bytes=68, n=n, a=1.5, x_off=64 * i, y_off=128)
    ctx.drain()
    for i, n in enumerate(ns):
        S, E = oracle.saxpy_tanh_sum(x[64 * i:64 * i + n], y[128:128 + n], 1.5)
        got = float(nout[128 * i + 64:128 * i + 68].view(np.float32)[0])
        assert abs(got - S) <= oracle.vec_tolerance(S, E)
    ctx.close()


@pytest.mark.parametrize("callback", ["event_poll", "event_chain", "event_blocking"])
def test_define_captured_templates_while_jobs_run(torch_gpu, callback):
    """Templates built by stream capture (a captured chain and a captured
    library call) are defined while another template's jobs are being
    launched onto the worker streams from two dispatcher threads.  The
    capture runs on the library's own stream, so no job launch is recorded
    into a new template and every job of every template completes correctly."""
    import threading
    _say("define captured templates while jobs run", callback)
    ctx = Context(mode="set", workers=4, slots=4, callback=callback, dispatchers=2)
    ta = ctx.define("box_hist", width=256, height=256, flags=0, copy="kernels")
    imgs = [synth.box_image(0, j) for j in range(16)]
    refs = [oracle.box_hist(im)[2] for im in imgs]
    n_a = 3000
    tin, nin = pinned(65536 * 16)
    for j, im in enumerate(imgs):
        nin[j * 65536:(j + 1) * 65536] = im.ravel()
    tout, nout = pinned(1152 * n_a)
    arr = ctx.job_array(n_a)
    idx = np.arange(n_a, dtype=np.uint64)
    arr["host_in"] = tin.data_ptr() + (idx % np.uint64(16)) * np.uint64(65536)
    arr["in_bytes"] = 65536
    arr["host_out"] = tout.data_ptr() + idx * np.uint64(1152)
    arr["out_bytes"] = 64 + 1024
    arr["user_tag"] = idx
    th = threading.Thread(target=lambda: ctx.submit_many(ta, arr))
    th.start()
    t0 = time.monotonic()
    while ctx.stats().completed < 50 and time.monotonic() - t0 < 30:
        time.sleep(0.001)
    tb = ctx.define("gauss_sobel", width=136, height=96, flags=A.SET_TF_CAPTURE, copy="kernels")
    tc = ctx.define("scan_lib", max_n=4097, copy="kernels")
    during = ctx.stats().completed
    th.join()
    assert during < n_a, "the definitions did not overlap the running jobs"
    g = [synth.normal_image(3, k, 96, 136) for k in range(4)]
    gin, gnin = pinned(4 * 96 * 136 * 4)
    gout, gnout = pinned(128 * 4)
    for k, im in enumerate(g):
        gnin[k * 4 * 96 * 136:(k + 1) * 4 * 96 * 136].view(np.float32)[:] = im.ravel()
        ctx.submit(tb, host_in=gin.data_ptr() + k * 4 * 96 * 136, in_bytes=4 * 96 * 136,
                   host_out=gout.data_ptr() + 128 * k, out_bytes=72)
    v = np.random.default_rng(4).integers(-(1 << 20), (1 << 20) + 1, 4097).astype(np.int32)
    sin, snin = pinned(4 * 4097)
    sout, snout = pinned(64 + 8 * 4097)
    snin.view(np.int32)[:] = v
    ctx.submit(tc, host_in=sin.data_ptr(), in_bytes=4 * 4097, host_out=sout.data_ptr(), out_bytes=64 + 8 * 4097)
    ctx.drain(timeout_ns=int(60e9))
    st = ctx.stats()
    assert st.completed == n_a + 5 and st.failed == 0
    out = nout.reshape(n_a, 1152)
    for i in range(n_a):
        _check_header(out[i], i, i)
        assert np.array_equal(out[i, 64:64 + 1024].view(np.uint32), refs[i % 16]), i
    for k, im in enumerate(g):
        ref = oracle.gauss_sobel(im, want_images=False)
        o = gnout[128 * k:128 * (k + 1)]
        assert abs(int(o[64:68].view(np.uint32)[0]) - ref["count"]) <= ref["band"]
        assert abs(float(o[68:72].view(np.float32)[0]) - ref["sum"]) <= 1e-5 * abs(ref["sum"])
    assert np.array_equal(snout[64:].view(np.int64), oracle.scan(v))
    ctx.close()


# ------------------------------------------------------------------ completion words in pinned host memory
@pytest.mark.parametrize("capture", [False, True])
def test_host_flag_completion_all_pipelines(torch_gpu, vec_pools, capture):
    """SET mode with the completion thread watching per-slot host words (no HIP
    call on the completion path): every pipeline, explicit and captured graphs."""
    _say("host_flag", "capture" if capture else "explicit")
    extra = A.SET_TF_CAPTURE if capture else 0
    imgs = [synth.box_image(0, j) for j in range(64)]
    outs, st = _run_images("set", "box_hist", imgs, np.uint8, flags=A.SET_TF_DEBUG | extra, callback="host_flag")
    for img, o in zip(imgs, outs):
        assert np.array_equal(o[64:64 + 1024].view(np.uint32), oracle.box_hist(img)[2])
    assert st.completed == 64
    g = [synth.normal_image(0, k) for k in range(4)]
    outs, _ = _run_images("set", "gauss_sobel", g + g, np.float32, workers=8, slots=4, flags=extra,
                          callback="host_flag")
    for k, img in enumerate(g + g):
        ref = oracle.gauss_sobel(img, want_images=False)
        assert abs(int(outs[k][64:68].view(np.uint32)[0]) - ref["count"]) <= ref["band"]
        assert abs(float(outs[k][68:72].view(np.float32)[0]) - ref["sum"]) <= 1e-5 * abs(ref["sum"])
    x, y = vec_pools[0], vec_pools[1]
    ns = np.array([1, 5, 1024, 4097, 65549, 1 << 20], np.int64)
    rng = np.random.default_rng(9)
    xo = 64 * rng.integers(0, (len(x) - ns) // 64)
    yo = 64 * rng.integers(0, (len(y) - ns) // 64)
    av = rng.uniform(0.5, 2, len(ns)).astype(np.float32)
    got, _ = _run_vec("set", vec_pools, np.concatenate([ns] * 8), np.concatenate([xo] * 8),
                      np.concatenate([yo] * 8), np.concatenate([av] * 8), callback="host_flag")
    for i, n in enumerate(ns):
        S, E = oracle.saxpy_tanh_sum(x[xo[i]:xo[i] + n], y[yo[i]:yo[i] + n], av[i])
        for r in range(8):
            assert abs(got[r * len(ns) + i] - S) <= oracle.vec_tolerance(S, E), (n, r)
    inputs = [synth.scan_input(0, k, n) for k, n in enumerate([1, 2047, 2048, 100003, 1 << 20])]
    res = _run_scan("set", inputs, max_n=1 << 20, extra_flags=extra, callback="host_flag")
    for v, r in zip(inputs, res):
        assert np.array_equal(r, oracle.scan(v))


@pytest.mark.parametrize("copy", ["kernels", "async_in", "nodes"])
def test_captured_thermal_and_vector_batch_templates(torch_gpu, vec_pools, copy):
    """Stream-captured templates of the two pipelines the capture tests above
    leave out: the thermal grid (a chain of 5 step kernels) matches the explicit
    template bit for bit and the oracle within its bound; batched vector jobs
    through a captured template match the explicit one bit for bit."""
    _say("captured thermal / vector batch", copy)
    grids = [synth.hotspot_input(4, k, 97, 132) for k in range(6)]
    a = _run_hotspot("set", grids, 5, copy=copy, flags=A.SET_TF_CAPTURE)
    b = _run_hotspot("set", grids, 5, copy=copy)
    for (t0, p), x, y in zip(grids, a, b):
        assert np.array_equal(x, y)
        ref = oracle.hotspot(t0, p, 5)
        assert np.max(np.abs(x - ref)) <= oracle.hotspot_tolerance(ref, 5)
    if copy == "nodes":
        return
    x, y, xd, yd = vec_pools
    js = synth.vec_jobs(8, 150, pool_len=len(x))
    jobs = np.zeros(150, dtype=A.VEC_JOB_DTYPE)
    for f in ("n", "a", "x_off", "y_off"):
        jobs[f] = js[f]
    res = []
    for flags in (A.SET_TF_CAPTURE, 0):
        ctx = Context(mode="set", workers=4, slots=2)
        tid = ctx.define("saxpy_batch", max_n=1 << 22, x_pool=xd, y_pool=yd, batch_max=16, tiles_max=1024,
                         flags=flags, copy=copy)
        r, _ = ctx.run_vector_jobs(tid, jobs)
        res.append(r)
        ctx.close()
    assert np.array_equal(res[0].view(np.uint32), res[1].view(np.uint32))
    for i in range(0, 150, 25):
        n, xo, yo = int(jobs["n"][i]), int(jobs["x_off"][i]), int(jobs["y_off"][i])
        S, E = oracle.saxpy_tanh_sum(x[xo:xo + n], y[yo:yo + n], jobs["a"][i])
        assert abs(float(res[0][i]) - S) <= oracle.vec_tolerance(S, E)


# ------------------------------------------------------------------ input copied ahead of the graph
@pytest.mark.parametrize("mode", ["sync", "graph", "batch", "queue", "set"])
def test_async_input_copy_all_modes(torch_gpu, vec_pools, mode):
    """SET_COPY_ASYNC_IN: the input goes by hipMemcpyAsync before the job's graph, the output by copy
    kernel inside it; results as with the other copy mechanisms."""
    _say("async input", mode)
    imgs = [synth.box_image(0, j, 37, 201) for j in range(6)]
    outs, _ = _run_images(mode, "box_hist", imgs, np.uint8, copy="async_in")
    for img, o in zip(imgs, outs):
        assert np.array_equal(o[64:64 + 1024].view(np.uint32), oracle.box_hist(img)[2])
    big = [synth.normal_image(0, k) for k in range(2)]
    outs, _ = _run_images(mode, "gauss_sobel", big, np.float32, workers=4, slots=4, flags=0, copy="async_in")
    for img, o in zip(big, outs):
        ref = oracle.gauss_sobel(img, want_images=False)
        assert abs(int(o[64:68].view(np.uint32)[0]) - ref["count"]) <= ref["band"]
        assert abs(float(o[68:72].view(np.float32)[0]) - ref["sum"]) <= 1e-5 * abs(ref["sum"])
    rng = np.random.default_rng(12)
    ins = [rng.integers(-(1 << 20), (1 << 20) + 1, n).astype(np.int32) for n in (1, 5, 4097, 1 << 21)]
    for v, r in zip(ins, _run_scan(mode, ins, max_n=1 << 21, copy="async_in")):
        assert np.array_equal(r, oracle.scan(v))
    if mode == "set":
        for v, r in zip(ins, _run_scan(mode, ins, max_n=1 << 21, copy="async_in", extra_flags=A.SET_TF_CAPTURE,
                                       callback="host_flag")):
            assert np.array_equal(r, oracle.scan(v))
        x, y, xd, yd = vec_pools
        js = synth.vec_jobs(3, 64, pool_len=len(x))
        jobs = np.zeros(64, dtype=A.VEC_JOB_DTYPE)
        for f in ("n", "a", "x_off", "y_off"):
            jobs[f] = js[f]
        ctx = Context(mode="set", workers=4, slots=4)
        tid = ctx.define("saxpy_batch", max_n=1 << 22, x_pool=xd, y_pool=yd, batch_max=16, tiles_max=512,
                         copy="async_in")
        res, nb = ctx.run_vector_jobs(tid, jobs)
        ctx.close()
        assert nb >= 4
        for i in range(64):
            n, xo, yo = int(jobs["n"][i]), int(jobs["x_off"][i]), int(jobs["y_off"][i])
            S, E = oracle.saxpy_tanh_sum(x[xo:xo + n], y[yo:yo + n], jobs["a"][i])
            assert abs(res[i] - S) <= oracle.vec_tolerance(S, E)


@pytest.mark.parametrize("mode", ["sync", "graph", "batch", "queue", "set"])
@pytest.mark.parametrize("copy_streams", [1, 3])
def test_async_input_copy_streams(torch_gpu, mode, copy_streams):
    """Input copies on library-owned copy streams (worker w on stream w % C, 3 of them not dividing the 8
    workers): every job still reads its own input, with slots reused many times over."""
    _say("input copy streams", mode, copy_streams)
    imgs = [synth.box_image(1, j, 64, 96) for j in range(40)]
    outs, _ = _run_images(mode, "box_hist", imgs, np.uint8, workers=8, slots=2, flags=0, copy="async_in",
                          input_copy_streams=copy_streams, callback="host_flag", dispatchers=2)
    for img, o in zip(imgs, outs):
        assert np.array_equal(o[64:64 + 1024].view(np.uint32), oracle.box_hist(img)[2])
    big = [synth.normal_image(1, k) for k in range(3)]
    outs, _ = _run_images(mode, "gauss_sobel", big * 4, np.float32, workers=8, slots=2, flags=0, copy="async_in",
                          input_copy_streams=copy_streams)
    for k, o in enumerate(outs):
        ref = oracle.gauss_sobel(big[k % 3], want_images=False)
        assert abs(int(o[64:68].view(np.uint32)[0]) - ref["count"]) <= ref["band"]
        assert abs(float(o[68:72].view(np.float32)[0]) - ref["sum"]) <= 1e-5 * abs(ref["sum"])
    for k in range(3):
        assert np.array_equal(outs[k][64:72], outs[k + 9][64:72])
    rng = np.random.default_rng(13)
    ins = [rng.integers(-(1 << 20), (1 << 20) + 1, n).astype(np.int32) for n in (3, 4097, 1 << 20)] * 3
    for v, r in zip(ins, _run_scan(mode, ins, max_n=1 << 20, copy="async_in", input_copy_streams=copy_streams)):
        assert np.array_equal(r, oracle.scan(v))


@pytest.mark.parametrize("callback", ["event_poll", "host_flag", "event_blocking"])
def test_prefetched_input_with_stealing(torch_gpu, callback):
    """SET with input-copy streams issues each input copy at bind.  With every job submitted to worker 0's
    queue, thieves retarget prefetched jobs (their copy is redone on the thief's stream) and the victim's
    slot takes a new job while the abandoned copy may still be landing: every result must still match."""
    _say("prefetched input + stealing", callback)
    imgs = [synth.box_image(2, j, 128, 128) for j in range(64)]
    outs, st = _run_images("set", "box_hist", imgs, np.uint8, workers=4, slots=4, flags=0, copy="async_in",
                           input_copy_streams=2, submit_policy=A.SET_SUBMIT_SKEW0, callback=callback,
                           dispatchers=4, inflight=1)
    for img, o in zip(imgs, outs):
        assert np.array_equal(o[64:64 + 1024].view(np.uint32), oracle.box_hist(img)[2])
    assert st.stolen > 0
    rng = np.random.default_rng(14)
    ins = [rng.integers(-(1 << 20), (1 << 20) + 1, n).astype(np.int32) for n in (7, 4096, 100003)] * 8
    for v, r in zip(ins, _run_scan("set", ins, max_n=1 << 17, copy="async_in", input_copy_streams=2,
                                   submit_policy=A.SET_SUBMIT_SKEW0, callback=callback, dispatchers=4)):
        assert np.array_equal(r, oracle.scan(v))


def test_prefetch_stale_copy_under_steals(torch_gpu):
    """Regression: a job stolen before launch leaves its prefetched copy queued behind one backlogged
    input-copy stream; a stolen job later bound to that slot copies on its own stream and must wait for
    the abandoned copy, or the abandoned copy lands on top of its input.  8 workers x 16 slots, 4 MiB
    inputs, one input-copy stream, 3 of 4 jobs hinted onto workers 0-3 so the others drain and steal
    in every direction; every job's result is checked."""
    _say("prefetch stale copy under steals")
    P, J = 8, 480
    imgs = [synth.normal_image(5, k) for k in range(P)]
    refs = [oracle.gauss_sobel(im, want_images=False) for im in imgs]
    ctx = Context(mode="set", workers=8, slots=16, inflight=1, input_copy_streams=1, callback="event_poll",
                  dispatchers=4)
    tid = ctx.define("gauss_sobel", width=1024, height=1024, flags=0, copy="async_in")
    ib, ob = ctx.in_bytes(tid), ctx.out_bytes(tid)
    tin, nin = pinned(ib * P)
    for k in range(P):
        nin[k * ib:(k + 1) * ib].view(np.float32)[:] = imgs[k].ravel()
    tout, nout = pinned(128 * J)
    arr = ctx.job_array(J)
    j = np.arange(J, dtype=np.uint64)
    arr["host_in"] = tin.data_ptr() + (j % np.uint64(P)) * np.uint64(ib)
    arr["in_bytes"] = ib
    arr["host_out"] = tout.data_ptr() + j * np.uint64(128)
    arr["out_bytes"] = ob
    arr["user_tag"] = j
    arr["worker_hint"] = np.where(j % 4 == 3, 4 + (j // 4) % 4, (j // 4) % 4).astype(np.int32)
    first = ctx.submit_many(tid, arr)
    ctx.drain()
    st = ctx.stats()
    ctx.close()
    out = nout.reshape(J, 128)
    bad = []
    for i in range(J):
        _check_header(out[i], first + i, i)
        r = refs[i % P]
        if abs(int(out[i, 64:68].view(np.uint32)[0]) - r["count"]) > r["band"] or \
                abs(float(out[i, 68:72].view(np.float32)[0]) - r["sum"]) > 1e-5 * abs(r["sum"]):
            bad.append(i)
    assert not bad, bad[:20]
    assert st.stolen > 0


# ------------------------------------------------------------------ library call captured into the job graph
@pytest.mark.parametrize("mode,copy,callback", [("set", "kernels", "host_flag"), ("set", "async_in", "event_poll"),
                                                ("set", "async_in", "event_blocking"),
                                                ("set", "nodes", "host_flag"), ("graph", "kernels", "host_flag"),
                                                ("queue", "kernels", "host_flag"), ("sync", "kernels", "host_flag")])
def test_library_scan_template(torch_gpu, mode, copy, callback):
    """rocPRIM's device scan captured between the job's begin/end kernels: exact int64 prefix sums,
    headers published, any slot, repeated replays of every slot's graph."""
    _say("library scan", mode, copy, callback)
    for n in (1, 1000, 1 << 21):
        inputs = [synth.scan_input(1, k, n) for k in range(3)]
        res = _run_scan(mode, inputs * 4, max_n=n, copy=copy, callback=callback, pipeline="scan_lib")
        for k, r in enumerate(res):
            assert np.array_equal(r, oracle.scan(inputs[k % 3])), (n, k)


def test_library_scan_stage_timing(torch_gpu):
    """The library stage is timed like the kernel stages."""
    ctx = Context(mode="set", workers=1, slots=2)
    tid = ctx.define("scan_lib", max_n=1 << 21)
    ib, ob = ctx.in_bytes(tid), ctx.out_bytes(tid)
    tin, nin = pinned(ib)
    nin.view(np.int32)[:] = synth.scan_input(1, 0, 1 << 21)
    tout, nout = pinned(ob)
    ctx.submit(tid, host_in=tin.data_ptr(), in_bytes=ib, host_out=tout.data_ptr(), out_bytes=ob)
    ctx.drain()
    names = [nm for nm, _ in ctx.stage_info(tid)]
    us = [ctx.time_stage(tid, i, 0, 5) for i in range(len(names))]
    ctx.close()
    assert names == ["job_begin", "scan_lib_rocprim", "job_end"]
    assert all(u > 0 for u in us)
    assert np.array_equal(nout[64:].view(np.int64), oracle.scan(synth.scan_input(1, 0, 1 << 21)))


# ------------------------------------------------------------------ thermal grid (iterative stencil)
def _run_hotspot(mode, grids, steps, workers=4, slots=4, copy="kernels", flags=0, **kw):
    h, w = grids[0][0].shape
    ctx = Context(mode=mode, workers=workers, slots=slots, **kw)
    tid = ctx.define("hotspot", width=w, height=h, max_n=steps, copy=copy, flags=flags)
    ib, ob = ctx.in_bytes(tid), ctx.out_bytes(tid)
    assert ib == 8 * h * w and ob == 64 + 4 * h * w
    istride, ostride = _up64(ib), _up64(ob)
    tin, nin = pinned(istride * len(grids))
    tout, nout = pinned(ostride * len(grids))
    for i, (t0, p) in enumerate(grids):
        nin[i * istride:i * istride + ib].view(np.float32)[:] = np.concatenate([t0.ravel(), p.ravel()])
    arr = ctx.job_array(len(grids))
    arr["host_in"] = tin.data_ptr() + np.arange(len(grids), dtype=np.uint64) * istride
    arr["in_bytes"] = ib
    arr["host_out"] = tout.data_ptr() + np.arange(len(grids), dtype=np.uint64) * ostride
    arr["out_bytes"] = ob
    first = ctx.submit_many(tid, arr)
    ctx.drain()
    ctx.close()
    outs = []
    for i in range(len(grids)):
        o = nout[i * ostride:(i + 1) * ostride]
        _check_header(o, first + i)
        outs.append(o[64:64 + 4 * h * w].view(np.float32).reshape(h, w).copy())
    return outs


HOT_SHAPES = [(1, 1), (1, 4), (3, 8), (5, 5), (33, 17), (17, 260), (64, 64), (70, 516), (256, 256)]


@pytest.mark.parametrize("mode", ["sync", "set"])
@pytest.mark.parametrize("shape", HOT_SHAPES)
def test_hotspot_parity(torch_gpu, mode, shape):
    _say("hotspot", mode, shape)
    h, w = shape
    grids = [synth.hotspot_input(0, k, h, w) for k in range(3)]
    for steps in (1, 7):
        outs = _run_hotspot(mode, grids, steps)
        for (t0, p), o in zip(grids, outs):
            ref = oracle.hotspot(t0, p, steps)
            assert np.max(np.abs(o - ref)) <= oracle.hotspot_tolerance(ref, steps), (shape, steps)


@pytest.mark.parametrize("shape", [(1024, 1024), (1030, 1028)])
def test_hotspot_parity_large_grids(torch_gpu, shape):
    """Grids of a million cells and more: full width, and a width with lanes
    past the edge and a ragged last row group."""
    _say("hotspot large", shape)
    h, w = shape
    grids = [synth.hotspot_input(1, k, h, w) for k in range(2)]
    for steps in (1, 3):
        outs = _run_hotspot("set", grids, steps, workers=2, slots=2)
        for (t0, p), o in zip(grids, outs):
            ref = oracle.hotspot(t0, p, steps)
            assert np.max(np.abs(o - ref)) <= oracle.hotspot_tolerance(ref, steps), (shape, steps)


@pytest.mark.parametrize("shape", [(37, 2048), (9, 4096), (3, 6144), (130, 2048),
                                   (2048, 2048), (1025, 4096), (683, 6144), (4097, 4096)])
def test_hotspot_parity_wide_grids(torch_gpu, shape):
    """Widths that are multiples of 2048, 1 and 3 steps.  Below 2^22 cells the
    window kernel; from 2^22 to 2^24 cells the row bands, 8 rows (2048^2) or
    16 (the others, ragged against the 16 rows, one to three 2048-column
    blocks per band); 4097x4096, above 2^24, the window kernel again."""
    _say("hotspot wide", shape)
    h, w = shape
    grids = [synth.hotspot_input(2, k, h, w) for k in range(2)]
    for steps in (1, 3):
        outs = _run_hotspot("set", grids, steps, workers=2, slots=2)
        for (t0, p), o in zip(grids, outs):
            ref = oracle.hotspot(t0, p, steps)
            assert np.max(np.abs(o - ref)) <= oracle.hotspot_tolerance(ref, steps), (shape, steps)


def test_tallest_image_and_grid(torch_gpu):
    """The tallest templates allowed, 2^19 rows of 4 columns: the second
    launch-grid dimension reaches 32,768 blocks for the image stages and
    65,536, its limit, for the thermal step (8 rows per block).  Every pixel
    of blur and mask, and every cell after 2 steps."""
    h, w = 1 << 19, 4
    _say("tallest image", h, w)
    img = synth.normal_image(7, 0, h, w)
    outs, _ = _run_images("set", "gauss_sobel", [img], np.float32, workers=1, slots=1)
    _check_gauss(img, outs[0])
    _say("tallest thermal grid", h, w)
    grids = [synth.hotspot_input(7, 0, h, w)]
    o = _run_hotspot("set", grids, 2, workers=1, slots=1)[0]
    ref = oracle.hotspot(grids[0][0], grids[0][1], 2)
    assert np.max(np.abs(o - ref)) <= oracle.hotspot_tolerance(ref, 2)


@pytest.mark.parametrize("mode", ["sync", "graph", "batch", "queue", "set"])
def test_hotspot_workload(torch_gpu, mode):
    """256x256 grids, 16 steps per job, 8 workers: every mode, identical results for identical inputs."""
    _say("hotspot workload", mode)
    grids = [synth.hotspot_input(0, k) for k in range(5)]
    outs = _run_hotspot(mode, grids * 4, 16, workers=8, slots=8, callback="host_flag", dispatchers=4)
    for i, o in enumerate(outs):
        t0, p = grids[i % 5]
        if i < 5:
            ref = oracle.hotspot(t0, p, 16)
            assert np.max(np.abs(o - ref)) <= oracle.hotspot_tolerance(ref, 16)
        assert np.array_equal(o, outs[i % 5])


@pytest.mark.parametrize("shape", [(256, 256), (97, 130)])
def test_hotspot_32_steps_within_1e5_relative(torch_gpu, shape):
    """The longest chain a template allows (32 steps) on seeded random grids,
    held to the 1e-5 relative bar for float32 stages itself: max |T_gpu -
    T_ref| <= 1e-5 max |T_ref|, tighter than the derived worst-case bound
    (33 * 8 * 2^-24 = 1.6e-5 relative) at this length."""
    _say("hotspot 32 steps, 1e-5 relative", shape)
    h, w = shape
    grids = [synth.hotspot_input(3, k, h, w) for k in range(4)]
    outs = _run_hotspot("set", grids, 32)
    for (t0, p), o in zip(grids, outs):
        ref = oracle.hotspot(t0, p, 32)
        err = float(np.max(np.abs(o.astype(np.float64) - ref)))
        _say("hotspot 32 steps", shape, "max error relative to max|T|: %.3g" % (err / float(np.max(np.abs(ref)))))
        assert err <= 1e-5 * float(np.max(np.abs(ref))), (shape, err)


def test_hotspot_pins_on_gpu(torch_gpu):
    """Ambient grid without power stays exactly ambient; 32 steps (the most a template allows)."""
    h, w = 40, 72
    amb = (np.full((h, w), 300.0, np.float32), np.zeros((h, w), np.float32))
    o = _run_hotspot("set", [amb], 32)[0]
    assert np.all(o == np.float32(300.0))


# ------------------------------------------------------------------ the benchmark's configurations at full size
BENCH_DMA = dict(callback="event_poll", inflight=1)


@pytest.mark.parametrize("callback", ["event_poll", "event_chain", "event_blocking"])
def test_bench_config_images_full_size(torch_gpu, callback):
    """1024^2 images as the benchmark runs them: 8 workers x 16 slots, DMA input copies, one job in flight per
    worker, one dispatcher thread, each completion mechanism the benchmark compares; 24 jobs over 8 images,
    each image's result identical in every slot it ran in."""
    _say("bench config: images 1024^2", callback)
    imgs = [synth.normal_image(0, k) for k in range(8)]
    outs, _ = _run_images("set", "gauss_sobel", imgs * 3, np.float32, workers=8, slots=16, flags=0,
                          copy="async_in", dispatchers=1, callback=callback, inflight=1)
    for k, o in enumerate(outs):
        ref = oracle.gauss_sobel(imgs[k % 8], want_images=False)
        assert abs(int(o[64:68].view(np.uint32)[0]) - ref["count"]) <= ref["band"]
        assert abs(float(o[68:72].view(np.float32)[0]) - ref["sum"]) <= 1e-5 * abs(ref["sum"])
        assert np.array_equal(o[64:72], outs[k % 8][64:72])


def test_bench_config_scan_full_size(torch_gpu):
    """2^21-element scans as the benchmark runs them: 8 workers x 4 slots, DMA input copies, one job in flight
    per worker, event polling, 4 dispatcher threads, stealing on."""
    _say("bench config: scan 2^21")
    inputs = [synth.scan_input(0, k) for k in range(4)] * 3
    res = _run_scan("set", inputs, max_n=1 << 21, workers=8, slots=4, copy="async_in", dispatchers=4, **BENCH_DMA)
    for v, r in zip(inputs, res):
        assert np.array_equal(r, oracle.scan(v))


@pytest.mark.parametrize("side,dispatchers", [(256, 2), (512, 1)])
def test_bench_config_hotspot_full_size(torch_gpu, side, dispatchers):
    """Thermal grids as the benchmark runs them: 16 steps, 8 workers x 16 slots, DMA input copies, one job in
    flight per worker, event polling, 2 dispatcher threads at 256^2 and 1 at 512^2."""
    _say("bench config: hotspot", side)
    grids = [synth.hotspot_input(0, k, side, side) for k in range(4)]
    outs = _run_hotspot("set", grids * 4, 16, workers=8, slots=16, copy="async_in", dispatchers=dispatchers,
                        **BENCH_DMA)
    for i, o in enumerate(outs):
        if i < 4:
            t0, p = grids[i]
            ref = oracle.hotspot(t0, p, 16)
            assert np.max(np.abs(o - ref)) <= oracle.hotspot_tolerance(ref, 16)
        assert np.array_equal(o, outs[i % 4])
