"""CPU oracle of every job's stage chain (ctypes wrapper over oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP path and never imports the product package.

Each function applies one job's whole stage chain to one job's input, in
plain loops and float64, and returns what that job must deliver (the method is
a scheduler, so every scheduled result must equal this, Sections 4.1-4.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BAND_EPS = 1e-5


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc -O2 (plain C, no vectorisation hints)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        _lib.oracle_box_hist_u8.argtypes = [P, I64, I64, P, P, P]
        _lib.oracle_gauss_taps.argtypes = [P]
        _lib.oracle_gauss_sobel_f32.argtypes = [P, I64, I64, ctypes.c_double, P, P, P, P, P, P]
        _lib.oracle_saxpy_tanh_sum_f32.argtypes = [P, P, I64, ctypes.c_float, P, P]
        _lib.oracle_scan_i32_i64.argtypes = [P, I64, P]
        _lib.oracle_hotspot_f32.argtypes = [P, P, I64, I64, ctypes.c_int, P]
        for f in ("oracle_box_hist_u8", "oracle_gauss_sobel_f32", "oracle_saxpy_tanh_sum_f32", "oracle_scan_i32_i64",
                  "oracle_hotspot_f32"):
            getattr(_lib, f).restype = ctypes.c_int
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise ValueError("%s failed with %d" % (what, rc))


def box_hist(img: np.ndarray):
    """3x3 zero-padded box sum S (uint16), Q = floor(S/9) (uint8), 256-bin histogram H (uint32)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    h, w = img.shape
    S = np.empty((h, w), np.uint16)
    Q = np.empty((h, w), np.uint8)
    H = np.empty(256, np.uint32)
    _check(lib().oracle_box_hist_u8(_ptr(img), h, w, _ptr(S), _ptr(Q), _ptr(H)), "box_hist")
    return S, Q, H


def gauss_taps() -> np.ndarray:
    g = np.empty(5, np.float64)
    lib().oracle_gauss_taps(_ptr(g))
    return g


def gauss_sobel(img: np.ndarray, band_eps: float = BAND_EPS, want_images: bool = True):
    """Returns dict: blur, mag (float64 images), mask (uint8), count (int), sum (float), band (int)."""
    img = np.ascontiguousarray(img, dtype=np.float32)
    h, w = img.shape
    blur = np.empty((h, w), np.float64) if want_images else None
    mag = np.empty((h, w), np.float64) if want_images else None
    mask = np.empty((h, w), np.uint8) if want_images else None
    cnt = np.zeros(1, np.uint32)
    s = np.zeros(1, np.float64)
    band = np.zeros(1, np.uint32)
    _check(lib().oracle_gauss_sobel_f32(_ptr(img), h, w, band_eps, _ptr(blur), _ptr(mag), _ptr(mask),
                                        _ptr(cnt), _ptr(s), _ptr(band)), "gauss_sobel")
    return {"blur": blur, "mag": mag, "mask": mask, "count": int(cnt[0]), "sum": float(s[0]), "band": int(band[0])}


def saxpy_tanh_sum(x: np.ndarray, y: np.ndarray, a: float):
    """S = sum tanh(a*x + y) in float64 and its float32 error allowance E."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    assert x.shape == y.shape
    S = np.zeros(1, np.float64)
    E = np.zeros(1, np.float64)
    _check(lib().oracle_saxpy_tanh_sum_f32(_ptr(x), _ptr(y), x.size, float(np.float32(a)), _ptr(S), _ptr(E)),
           "saxpy_tanh_sum")
    return float(S[0]), float(E[0])


def scan(x: np.ndarray) -> np.ndarray:
    """Inclusive prefix sum of int32 into int64."""
    x = np.ascontiguousarray(x, dtype=np.int32)
    out = np.empty(x.size, np.int64)
    _check(lib().oracle_scan_i32_i64(_ptr(x), x.size, _ptr(out)), "scan")
    return out


HOTSPOT = {"cx": 0.1, "cy": 0.1, "cz": 1.0 / 640.0, "cp": 0.5, "t_amb": 300.0}


def hotspot(T0: np.ndarray, P: np.ndarray, iters: int) -> np.ndarray:
    """Temperature grid after `iters` explicit heat steps (float64)."""
    T0 = np.ascontiguousarray(T0, dtype=np.float32)
    P = np.ascontiguousarray(P, dtype=np.float32)
    assert T0.shape == P.shape and T0.ndim == 2
    out = np.empty(T0.shape, np.float64)
    _check(lib().oracle_hotspot_f32(_ptr(T0), _ptr(P), T0.shape[0], T0.shape[1], int(iters), _ptr(out)), "hotspot")
    return out


def hotspot_tolerance(ref: np.ndarray, iters: int) -> float:
    """Allowed max |T_gpu - T_ref| for float32 evaluation: each step rounds a
    handful of operations on values of magnitude <= max|T| (the coefficients
    sum below 1), and the monotone step does not amplify earlier errors, so
    the error grows at most linearly: (iters + 1) * 8 * 2^-24 * max|T|."""
    return (iters + 1) * 8.0 * 2.0 ** -24 * float(np.max(np.abs(ref)))


def vec_tolerance(S_ref: float, E: float) -> float:
    """Allowed |S_gpu - S_ref| for the cancelling float32 sum: max(1e-5 |S_ref|, E)."""
    return max(1e-5 * abs(S_ref), E)


def vec_verdict(S_gpu: float, S_ref: float, E: float):
    """(passes, by_floor): whether S_gpu is within vec_tolerance, and whether it
    passes only because of the floor E (its error is above 1e-5 |S_ref|).  The
    share of jobs decided by the floor is what the loose bound lets through."""
    err = abs(float(S_gpu) - S_ref)
    ok = err <= vec_tolerance(S_ref, E)
    return ok, bool(ok and err > 1e-5 * abs(S_ref))
