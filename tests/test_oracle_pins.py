"""Pins of the CPU oracle against facts it does not compute itself.

Each pin is written independently of oracle.c: brute force in a different
formulation (padded shifted sums, direct 2-D 5x5 convolution, math.fsum),
closed forms, and invariants (symmetry, reflection, transpose).  A plausible
slip in the oracle (dropped term, wrong sign or index, transposed kernel, wrong
border rule, wrong divisor) fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ----------------------------------------------------------------- box / histogram
def _box_brute(img):
    """3x3 zero-padded sum as nine shifted views of a zero-padded copy."""
    h, w = img.shape
    p = np.zeros((h + 2, w + 2), np.int64)
    p[1:-1, 1:-1] = img
    s = sum(p[dy:dy + h, dx:dx + w] for dy in range(3) for dx in range(3))
    q = s // 9
    hist = np.bincount(q.ravel(), minlength=256)
    return s, q, hist


@pytest.mark.parametrize("h", range(1, 7))
@pytest.mark.parametrize("w", range(1, 7))
def test_box_brute_force_small(h, w, rng):
    for img in (rng.integers(0, 256, (h, w)), np.full((h, w), 255), np.zeros((h, w)),
                rng.choice([0, 255], (h, w))):
        img = img.astype(np.uint8)
        S, Q, H = oracle.box_hist(img)
        s, q, hist = _box_brute(img)
        assert np.array_equal(S, s)
        assert np.array_equal(Q, q)
        assert np.array_equal(H, hist)
        assert H.sum() == h * w


@pytest.mark.parametrize("c", [0, 1, 8, 9, 100, 200, 254, 255])
def test_box_constant_image_closed_form(c):
    h = w = 256
    S, Q, H = oracle.box_hist(np.full((h, w), c, np.uint8))
    expect = np.zeros(256, np.int64)
    expect[c] += (h - 2) * (w - 2)          # 64,516 interior pixels see 9 values
    expect[(6 * c) // 9] += 2 * (h - 2) + 2 * (w - 2)  # 1,016 edge pixels see 6
    expect[(4 * c) // 9] += 4               # 4 corners see 4
    assert np.array_equal(H, expect)
    assert int(H.sum()) == 65536


def test_box_all_255_values():
    _, Q, _ = oracle.box_hist(np.full((256, 256), 255, np.uint8))
    assert Q[1:-1, 1:-1].min() == 255 and Q[1:-1, 1:-1].max() == 255
    assert Q[0, 0] == Q[0, -1] == Q[-1, 0] == Q[-1, -1] == 113
    assert set(np.unique(Q[0, 1:-1])) == {170}
    assert set(np.unique(Q[1:-1, 0])) == {170}


def test_box_empty():
    S, Q, H = oracle.box_hist(np.zeros((0, 5), np.uint8))
    assert H.sum() == 0


# ----------------------------------------------------------------- Gaussian / Sobel
def _taps_independent():
    e = [math.exp(-k * k / 2.0) for k in (-2, -1, 0, 1, 2)]
    s = math.fsum(e)
    return [float(np.float32(v / s)) for v in e]


def test_gauss_taps_values_and_ratios():
    g = oracle.gauss_taps()
    assert list(g) == _taps_independent()
    assert g[0] == g[4] and g[1] == g[3]
    # ratios of a sigma=1 Gaussian: g(1)/g(0) = e^-1/2, g(2)/g(0) = e^-2, to float32 rounding
    assert abs(g[1] / g[2] - math.exp(-0.5)) < 2e-7
    assert abs(g[0] / g[2] - math.exp(-2.0)) < 2e-7
    assert abs(math.fsum(g) - 1.0) < 5 * 2 ** -24


def _gauss_sobel_brute(img):
    """Direct 2-D 5x5 convolution with weights g_i*g_j and replicated borders, then an
    explicit-neighbour Sobel; pure Python loops over tiny images."""
    g = _taps_independent()
    h, w = img.shape
    cl = lambda v, n: min(max(v, 0), n - 1)
    blur = [[0.0] * w for _ in range(h)]
    for y in range(h):
        for x in range(w):
            terms = []
            for i in range(5):
                for j in range(5):
                    terms.append(g[i] * g[j] * float(img[cl(y + i - 2, h)][cl(x + j - 2, w)]))
            blur[y][x] = math.fsum(terms)
    mag = np.zeros((h, w))
    for y in range(h):
        for x in range(w):
            B = lambda dy, dx: blur[cl(y + dy, h)][cl(x + dx, w)]
            gx = (B(-1, 1) + 2 * B(0, 1) + B(1, 1)) - (B(-1, -1) + 2 * B(0, -1) + B(1, -1))
            gy = (B(1, -1) + 2 * B(1, 0) + B(1, 1)) - (B(-1, -1) + 2 * B(-1, 0) + B(-1, 1))
            mag[y, x] = math.hypot(gx, gy)
    return np.array(blur), mag


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (2, 2), (3, 5), (5, 3), (6, 6), (9, 11), (11, 9)])
def test_gauss_sobel_brute_force(shape, rng):
    img = (rng.standard_normal(shape) * 2).astype(np.float32)
    r = oracle.gauss_sobel(img)
    blur, mag = _gauss_sobel_brute(img)
    np.testing.assert_allclose(r["blur"], blur, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(r["mag"], mag, rtol=1e-11, atol=1e-12)
    assert np.array_equal(r["mask"], (mag > 1.0).astype(np.uint8))
    assert r["count"] == int((mag > 1.0).sum())
    assert abs(r["sum"] - math.fsum(mag.ravel())) <= 1e-11 * max(1.0, abs(r["sum"]))


def test_gauss_impulse_exact():
    """One 1.0 at least 2 pixels from every border blurs to exactly g_i * g_j."""
    g = oracle.gauss_taps()
    img = np.zeros((12, 13), np.float32)
    y0, x0 = 5, 6
    img[y0, x0] = 1.0
    b = oracle.gauss_sobel(img)["blur"]
    for i in range(5):
        for j in range(5):
            assert b[y0 + i - 2, x0 + j - 2] == g[i] * g[j]
    mask = np.ones_like(b, bool)
    mask[y0 - 2:y0 + 3, x0 - 2:x0 + 3] = False
    assert np.all(b[mask] == 0.0)


@pytest.mark.parametrize("c", [0.0, 1.0, -3.5, 1e3])
def test_gauss_sobel_constant_image(c):
    """Blur of a constant image is constant, so the gradient is zero up to double rounding."""
    r = oracle.gauss_sobel(np.full((17, 33), c, np.float32))
    assert r["count"] == 0
    assert r["sum"] <= 1e-14 * abs(c) * 17 * 33
    assert np.all(r["mag"] <= 1e-14 * abs(c))
    assert np.ptp(r["blur"]) <= 1e-15 * abs(c)


@pytest.mark.parametrize("alpha,above", [(0.25, True), (0.0625, False)])
def test_gauss_sobel_ramp(alpha, above):
    """I = alpha*x: interior blur = alpha*x*(sum g)^2, |grad| = 8*alpha*(sum g)^2."""
    g = oracle.gauss_taps()
    S2 = math.fsum(g) ** 2
    h, w = 9, 24
    img = (alpha * np.tile(np.arange(w, dtype=np.float64), (h, 1))).astype(np.float32)
    r = oracle.gauss_sobel(img)
    cols = slice(3, w - 3)
    np.testing.assert_allclose(r["blur"][:, 2:w - 2], (alpha * np.arange(2, w - 2) * S2)[None, :].repeat(h, 0),
                               rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r["mag"][:, cols], 8 * alpha * S2, rtol=1e-12)
    assert bool(np.all(r["mask"][:, cols] == (1 if above else 0)))


def test_gauss_sobel_transpose_and_reflection_invariance(rng):
    img = rng.standard_normal((23, 31)).astype(np.float32)
    r = oracle.gauss_sobel(img)
    rt = oracle.gauss_sobel(np.ascontiguousarray(img.T))
    rf = oracle.gauss_sobel(np.ascontiguousarray(img[:, ::-1]))
    np.testing.assert_allclose(rt["mag"], r["mag"].T, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(rf["mag"], r["mag"][:, ::-1], rtol=1e-12, atol=1e-12)


def test_gauss_sobel_band_counts_near_threshold():
    # a ramp whose magnitude is 1 up to rounding: every interior pixel lies in the band
    g = oracle.gauss_taps()
    S2 = math.fsum(g) ** 2
    alpha = np.float32(1.0 / (8 * S2))
    img = (alpha * np.tile(np.arange(16, dtype=np.float32), (6, 1))).astype(np.float32)
    r = oracle.gauss_sobel(img, band_eps=1e-5)
    assert r["band"] >= 6 * 10


def test_gauss_sobel_empty():
    r = oracle.gauss_sobel(np.zeros((0, 4), np.float32))
    assert r["count"] == 0 and r["sum"] == 0.0


# ----------------------------------------------------------------- vector job
def test_saxpy_brute_force(rng):
    for n in (1, 2, 3, 17, 64, 1000):
        x = rng.uniform(-1, 1, n).astype(np.float32)
        y = rng.uniform(-1, 1, n).astype(np.float32)
        a = np.float32(rng.uniform(0.5, 2))
        S, E = oracle.saxpy_tanh_sum(x, y, a)
        ref = math.fsum(math.tanh(float(a) * float(xi) + float(yi)) for xi, yi in zip(x, y))
        assert abs(S - ref) <= 1e-13 * max(1.0, n)
        depth = max(0, math.ceil(math.log2(n))) if n > 1 else 0
        z = [float(a) * float(xi) + float(yi) for xi, yi in zip(x, y)]
        t = [math.tanh(v) for v in z]
        Eref = 2 ** -24 * ((depth + 4) * math.fsum(abs(v) for v in t) + math.fsum(abs(v) for v in z))
        assert abs(E - Eref) <= 1e-12 * Eref


def test_saxpy_saturated_and_zero():
    n = 4097
    S, _ = oracle.saxpy_tanh_sum(np.ones(n, np.float32), np.zeros(n, np.float32), 16.0)
    assert abs(S - n * math.tanh(16.0)) < 1e-9 and abs(S - n) < 1e-9
    S0, E0 = oracle.saxpy_tanh_sum(np.zeros(n, np.float32), np.zeros(n, np.float32), 1.5)
    assert S0 == 0.0 and E0 == 0.0
    Se, _ = oracle.saxpy_tanh_sum(np.zeros(0, np.float32), np.zeros(0, np.float32), 1.0)
    assert Se == 0.0


def test_saxpy_ternary_saturated_sum_is_the_integer_sum(rng):
    """x in {-1, 0, 1}, a = 16, y = 0: tanh(+-16) is 1 - 2.5e-14 in magnitude,
    so S is the integer sum of x to within n * 2.5e-14 (the exact-sum pins of
    the device paths rely on float32 rounding that residue away)."""
    for n in (1, 3, 4097, 65549):
        x = rng.integers(-1, 2, n).astype(np.float32)
        S, _ = oracle.saxpy_tanh_sum(x, np.zeros(n, np.float32), 16.0)
        exact = int(np.sum(x.astype(np.int64)))
        assert abs(S - exact) <= n * 2.6e-14
        assert np.float32(S) == np.float32(exact)


def test_saxpy_floor_bounds_float32_evaluations(rng):
    """The floor E bounds the error of actual float32 evaluations: z and tanh
    rounded to float32, then summed sequentially, pairwise, in reverse and in
    blocks of 1024 partials; each stays within E of the float64 S."""
    for n in (7, 1000, 4096, 65549):
        x = rng.uniform(-1, 1, n).astype(np.float32)
        y = rng.uniform(-1, 1, n).astype(np.float32)
        a = np.float32(rng.uniform(0.5, 2))
        S, E = oracle.saxpy_tanh_sum(x, y, float(a))
        t = np.tanh(a * x + y).astype(np.float32)
        seq = np.cumsum(t, dtype=np.float32)[-1]
        pair = np.sum(t, dtype=np.float32)
        rev = np.cumsum(t[::-1], dtype=np.float32)[-1]
        blocks = np.sum(np.array([np.sum(t[k:k + 1024], dtype=np.float32) for k in range(0, n, 1024)],
                                 np.float32), dtype=np.float32)
        for v in (seq, pair, rev, blocks):
            assert abs(float(v) - S) <= E, (n, float(v), S, E)


def test_saxpy_odd_symmetry_and_a_zero(rng):
    x = rng.uniform(-1, 1, 5000).astype(np.float32)
    y = rng.uniform(-1, 1, 5000).astype(np.float32)
    S, _ = oracle.saxpy_tanh_sum(x, y, 1.25)
    Sn, _ = oracle.saxpy_tanh_sum(-x, -y, 1.25)
    assert Sn == -S
    S0, _ = oracle.saxpy_tanh_sum(x, y, 0.0)
    assert abs(S0 - math.fsum(math.tanh(float(v)) for v in y)) < 1e-10


def test_saxpy_uses_both_operands(rng):
    """a*x + y, not a*y + x or a*(x+y)."""
    x = np.array([0.5], np.float32)
    y = np.array([0.25], np.float32)
    S, _ = oracle.saxpy_tanh_sum(x, y, 2.0)
    assert S == math.tanh(2.0 * 0.5 + 0.25)


# ----------------------------------------------------------------- scan
def test_scan_closed_forms():
    n = 1 << 21
    c = 7
    assert np.array_equal(oracle.scan(np.full(n, c, np.int32)), c * np.arange(1, n + 1, dtype=np.int64))
    i = np.arange(n, dtype=np.int64)
    assert np.array_equal(oracle.scan(np.arange(n, dtype=np.int32)), i * (i + 1) // 2)
    big = oracle.scan(np.full(n, 1 << 20, np.int32))
    assert big[-1] == (1 << 20) * n == 1 << 41
    neg = oracle.scan(np.full(n, -(1 << 20), np.int32))
    assert neg[-1] == -(1 << 41)


def test_scan_brute_force(rng):
    for n in [0, 1, 2, 3, 5, 63, 64, 65, 1000, 1023, 1024]:
        x = rng.integers(-(1 << 20), (1 << 20) + 1, n).astype(np.int32)
        out = oracle.scan(x)
        acc, ref = 0, []
        for v in x.tolist():
            acc += v
            ref.append(acc)
        assert out.tolist() == ref


# ------------------------------------------------------------------ thermal grid
HS = oracle.HOTSPOT


def test_hotspot_ambient_is_a_fixed_point():
    T0 = np.full((7, 9), HS["t_amb"], np.float32)
    P = np.zeros((7, 9), np.float32)
    assert np.array_equal(oracle.hotspot(T0, P, 12), T0.astype(np.float64))


@pytest.mark.parametrize("t0,p,k", [(320.0, 0.0, 5), (300.0, 0.25, 9), (280.0, 1.0, 1), (350.0, 0.5, 0)])
def test_hotspot_uniform_closed_form(t0, p, k):
    # a uniform grid stays uniform (zero-flux borders, zero Laplacian); the
    # scalar recurrence T <- T + cp*p + cz*(Tamb - T) sums to a geometric series
    T0 = np.full((5, 6), t0, np.float32)
    P = np.full((5, 6), p, np.float32)
    fix = HS["t_amb"] + HS["cp"] * np.float64(np.float32(p)) / HS["cz"]
    want = fix + (np.float64(np.float32(t0)) - fix) * (1.0 - HS["cz"]) ** k
    got = oracle.hotspot(T0, P, k)
    assert np.allclose(got, want, rtol=0, atol=1e-9)


def _hotspot_brute(T0, P, k):
    # independent restatement: padded arrays instead of clamped indices
    T = T0.astype(np.float64)
    for _ in range(k):
        E = np.pad(T, 1, mode="edge")
        lap_y = E[:-2, 1:-1] + E[2:, 1:-1] - 2 * T
        lap_x = E[1:-1, :-2] + E[1:-1, 2:] - 2 * T
        T = T + HS["cp"] * P.astype(np.float64) + HS["cy"] * lap_y + HS["cx"] * lap_x + HS["cz"] * (HS["t_amb"] - T)
    return T


@pytest.mark.parametrize("shape,k", [((1, 1), 3), ((1, 5), 4), ((4, 1), 2), ((3, 4), 3), ((6, 7), 6)])
def test_hotspot_brute_force(shape, k, rng):
    T0 = (300 + 40 * rng.random(shape)).astype(np.float32)
    P = rng.random(shape).astype(np.float32)
    assert np.allclose(oracle.hotspot(T0, P, k), _hotspot_brute(T0, P, k), rtol=0, atol=1e-9)


def test_hotspot_symmetries_and_maximum_principle(rng):
    T0 = (300 + 50 * rng.random((8, 8))).astype(np.float32)
    P = np.zeros((8, 8), np.float32)
    out = oracle.hotspot(T0, P, 10)
    # cx == cy: transposing and flipping the input does the same to the output
    assert np.allclose(oracle.hotspot(T0.T.copy(), P, 10), out.T, rtol=0, atol=1e-9)
    assert np.allclose(oracle.hotspot(T0[::-1, ::-1].copy(), P, 10), out[::-1, ::-1], rtol=0, atol=1e-9)
    # no source: a monotone step keeps every cell within [min(T0, Tamb), max(T0, Tamb)]
    assert out.min() >= min(T0.min(), HS["t_amb"]) - 1e-9 and out.max() <= max(T0.max(), HS["t_amb"]) + 1e-9
    # a single hot cell spreads symmetrically and the heat above ambient decays by (1 - cz) per step
    T1 = np.full((9, 9), HS["t_amb"], np.float32)
    T1[4, 4] = 400.0
    o1 = oracle.hotspot(T1, P[:1, :1].repeat(9, 0).repeat(9, 1), 3)
    assert np.allclose(o1, o1.T, rtol=0, atol=1e-12) and np.allclose(o1, o1[::-1, :], rtol=0, atol=1e-12)
    assert (o1 - HS["t_amb"]).sum() == pytest.approx(100.0 * (1 - HS["cz"]) ** 3, rel=1e-12)
