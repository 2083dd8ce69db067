"""Seeded synthetic inputs for every job family.

This module only draws random numbers; it holds none of the pipeline arithmetic,
so both the HIP path and the CPU oracle can take their inputs from it.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014, in the public-domain form popularised by
Vigna).  Every object (an image, a vector job, a pool) owns one stream whose
initial state is ``seed + (cfg << 40) + k``; the i-th draw (i = 1, 2, ...) of a
stream is ``mix(state0 + i * GOLDEN)``, which lets numpy produce a whole stream
at once.

Job families (the paper measures throughput of many independent short jobs,
Section 5.1; the job shapes below are this implementation's synthetic stand-ins):

* cfg 0: 256x256 uint8 images, uniform 0..255, one stream per job id.
* cfg 1: 1024x1024 float32 images ~ N(0, 1) (Box-Muller), pool of 61.
* cfg 2: vector jobs; n log-uniform in [4096, 4194304), a ~ U[0.5, 2], window
  offsets into two device-resident U[-1, 1) pools of 2**27 floats.
* cfg 3: 2**21 int32 ~ U[-2**20, 2**20], pool of 31.
* cfg 4: serving mix; Poisson arrivals, image sides {256, 512, 1024, 2048}.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1

TWO_M24 = 2.0 ** -24
TWO_M53 = 2.0 ** -53

CFG_BOX = 0
CFG_IMAGE = 1
CFG_VECTOR = 2
CFG_SCAN = 3
CFG_SERVE = 4
CFG_HOTSPOT = 5

IMAGE_POOL = 61
SCAN_POOL = 31
VEC_POOL_LEN = 1 << 27
SERVE_SIDES = (256, 512, 1024, 2048)

# object index k of the two vector pools (outside any job id range)
_K_XPOOL = 1 << 39
_K_YPOOL = (1 << 39) + 1


def stream_key(seed: int, cfg: int, k: int) -> int:
    return (int(seed) + (int(cfg) << 40) + int(k)) & MASK64


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def draws(key: int, count: int, start: int = 0) -> np.ndarray:
    """Draws start+1 .. start+count of the stream with initial state `key`."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        st = np.uint64(key) + i * GOLDEN
    return _mix(st)


def draw_one(key: int, index: int) -> int:
    """The index-th draw (1-based) as a Python int (scalar reference form)."""
    z = (key + index * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


# ---------------------------------------------------------------- draw forms
def as_u8(z: np.ndarray) -> np.ndarray:
    return (z >> np.uint64(56)).astype(np.uint8)


def as_unit24(z: np.ndarray) -> np.ndarray:
    """k * 2**-24 for the top 24 bits, exact in float32 and float64."""
    return (z >> np.uint64(40)).astype(np.float64) * TWO_M24


def as_unit53(z: np.ndarray) -> np.ndarray:
    return (z >> np.uint64(11)).astype(np.float64) * TWO_M53


def as_sym_f32(z: np.ndarray) -> np.ndarray:
    """U[-1, 1) in float32 (exact: k * 2**-23 - 1)."""
    return (as_unit24(z) * 2.0 - 1.0).astype(np.float32)


def as_i32_range(z: np.ndarray, lo: int, hi: int) -> np.ndarray:
    span = np.uint64(hi - lo + 1)
    return ((z % span).astype(np.int64) + lo).astype(np.int32)


def normal_f32(key: int, count: int, chunk: int = 1 << 21) -> np.ndarray:
    """count N(0,1) float32 values: Box-Muller in float64, cosine branch only,
    draws (2i+1, 2i+2) feed value i."""
    out = np.empty(count, dtype=np.float32)
    for c0 in range(0, count, chunk):
        c = min(chunk, count - c0)
        z = draws(key, 2 * c, start=2 * c0)
        u1 = ((z[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * TWO_M53
        u2 = (z[1::2] >> np.uint64(11)).astype(np.float64) * TWO_M53
        out[c0:c0 + c] = (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).astype(np.float32)
    return out


# ---------------------------------------------------------------- families
def box_image(seed: int, job: int, h: int = 256, w: int = 256) -> np.ndarray:
    """cfg 0 image of job `job`: uniform uint8, stream key = seed + job id."""
    return as_u8(draws(stream_key(seed, CFG_BOX, job), h * w)).reshape(h, w)


def normal_image(seed: int, k: int, h: int = 1024, w: int = 1024, cfg: int = CFG_IMAGE) -> np.ndarray:
    """N(0,1) float32 image number k of family `cfg`."""
    return normal_f32(stream_key(seed, cfg, k), h * w).reshape(h, w)


def image_pool(seed: int, count: int = IMAGE_POOL, h: int = 1024, w: int = 1024, out=None) -> np.ndarray:
    """The cfg-1 pool: `count` images; job j uses entry j % count."""
    if out is None:
        out = np.empty((count, h, w), dtype=np.float32)
    for p in range(count):
        out[p] = normal_image(seed, p, h, w)
    return out


def serve_image_pool(seed: int, side: int, count: int = IMAGE_POOL, out=None) -> np.ndarray:
    si = SERVE_SIDES.index(side)
    if out is None:
        out = np.empty((count, side, side), dtype=np.float32)
    for p in range(count):
        out[p] = normal_image(seed, (si << 20) + p, side, side, cfg=CFG_SERVE)
    return out


def scan_input(seed: int, k: int, n: int = 1 << 21) -> np.ndarray:
    """cfg-3 input k: int32 uniform on [-2**20, 2**20]."""
    return as_i32_range(draws(stream_key(seed, CFG_SCAN, k), n), -(1 << 20), 1 << 20)


def hotspot_input(seed: int, k: int, h: int = 256, w: int = 256):
    """Thermal-grid input k: temperatures T0 uniform on [310, 340) K and a
    skewed power map P = 2 u^4 (u uniform on [0, 1)): a few hot cells on a cool
    background.  Returns (T0, P), float32 h x w each."""
    z = draws(stream_key(seed, CFG_HOTSPOT, k), 2 * h * w)
    t0 = (310.0 + 30.0 * as_unit24(z[: h * w])).astype(np.float32).reshape(h, w)
    u = as_unit24(z[h * w:]).astype(np.float64)
    p = (2.0 * u ** 4).astype(np.float32).reshape(h, w)
    return t0, p


def scan_pool(seed: int, count: int = SCAN_POOL, n: int = 1 << 21, out=None) -> np.ndarray:
    if out is None:
        out = np.empty((count, n), dtype=np.int32)
    for p in range(count):
        out[p] = scan_input(seed, p, n)
    return out


def vec_pool(seed: int, which: str, length: int = VEC_POOL_LEN, out=None, chunk: int = 1 << 22) -> np.ndarray:
    """Device-resident vector pool 'x' or 'y': U[-1, 1) float32."""
    key = stream_key(seed, CFG_VECTOR, _K_XPOOL if which == "x" else _K_YPOOL)
    if out is None:
        out = np.empty(length, dtype=np.float32)
    for c0 in range(0, length, chunk):
        c = min(chunk, length - c0)
        out[c0:c0 + c] = as_sym_f32(draws(key, c, start=c0))
    return out


VEC_N_MIN = 4096
VEC_N_SPAN = 1024.0  # n = floor(4096 * 1024**u), u in [0, 1)


def vec_jobs(seed: int, count: int, pool_len: int = VEC_POOL_LEN, first: int = 0, cfg: int = CFG_VECTOR,
             n_min: int = VEC_N_MIN, n_span: float = VEC_N_SPAN):
    """Per-job parameters of the vector family: dict of arrays n, a, x_off, y_off.

    Stream key = seed + (cfg << 40) + job id; draws 1..4 give n, a, x_off, y_off.
    Offsets are multiples of 64 elements with off + n <= pool_len."""
    n = np.empty(count, dtype=np.int64)
    a = np.empty(count, dtype=np.float32)
    xo = np.empty(count, dtype=np.int64)
    yo = np.empty(count, dtype=np.int64)
    base = np.arange(first, first + count, dtype=np.uint64)
    keys = (np.uint64(int(seed) & MASK64) + np.uint64(int(cfg) << 40) + base)
    with np.errstate(over="ignore"):
        z = [_mix(keys + np.uint64(i) * GOLDEN) for i in (1, 2, 3, 4)]
    u = as_unit53(z[0])
    n[:] = np.floor(n_min * np.power(n_span, u)).astype(np.int64)
    n[:] = np.minimum(n, int(n_min * n_span) - 1)
    a[:] = (0.5 + 1.5 * as_unit24(z[1])).astype(np.float32)
    ux = as_unit53(z[2])
    uy = as_unit53(z[3])
    xo[:] = 64 * np.floor(ux * (pool_len - n) / 64.0).astype(np.int64)
    yo[:] = 64 * np.floor(uy * (pool_len - n) / 64.0).astype(np.int64)
    return {"n": n, "a": a, "x_off": xo, "y_off": yo}


def poisson_arrivals(seed: int, rate_per_s: float, duration_s: float, max_count: int = 1 << 24) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson process: inter-arrival -ln(u)/rate."""
    key = stream_key(seed, CFG_SERVE, (1 << 39) + int(rate_per_s))
    est = int(rate_per_s * duration_s * 1.2) + 64
    est = min(est, max_count)
    z = draws(key, est)
    u = ((z >> np.uint64(11)).astype(np.float64) + 1.0) * TWO_M53
    t = np.cumsum(-np.log(u) / rate_per_s)
    return t[t < duration_s]


def serve_mix(seed: int, count: int):
    """Per-request kind of the serving mix: kind 0 = image (side index 0..3 in `side_idx`,
    pool entry `pool_idx`), kind 1 = vector job (parameters from vec_jobs with cfg 4)."""
    key = stream_key(seed, CFG_SERVE, (1 << 38))
    z = draws(key, 3 * count).reshape(count, 3)
    kind = (z[:, 0] >> np.uint64(63)).astype(np.int32)
    side_idx = (z[:, 1] >> np.uint64(62)).astype(np.int32)
    pool_idx = (z[:, 2] % np.uint64(IMAGE_POOL)).astype(np.int32)
    return {"kind": kind, "side_idx": side_idx, "pool_idx": pool_idx}
