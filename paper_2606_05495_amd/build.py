"""Build the native library libset.so in-tree (gfx950 device code via hipcc,
host-only C++ via g++), and the ThreadSanitizer scheduler test binary.

    python -m paper_2606_05495_amd.build          # incremental
    python -m paper_2606_05495_amd.build --force  # rebuild everything
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libset.so")
TSAN_BIN = os.path.join(OBJ, "sched_tsan_test")

ARCH = os.environ.get("SET_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_SOURCES = ["kernels.hip", "backend_hip.hip", "noalloc.hip", "lib_scan.hip"]
CPP_SOURCES = ["sched.cpp", "layout.cpp", "backend_fake.cpp"]
HEADERS = ["internal.hpp", "kernels.hpp", "tiles.hpp"]

# Packed fp32 instructions are switched off for all device code (the compiler
# would otherwise form them from ordinary float code).
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wextra", "-Wno-unused-parameter",
             "-pthread"]


def _deps_mtime() -> float:
    m = os.path.getmtime(os.path.join(INCLUDE, "set.h"))
    for h in HEADERS:
        m = max(m, os.path.getmtime(os.path.join(CSRC, h)))
    return m


def _stale(obj: str, src: str, force: bool) -> bool:
    if force or not os.path.exists(obj):
        return True
    return os.path.getmtime(obj) < max(os.path.getmtime(src), _deps_mtime())


def _run_all(cmds):
    procs = [(c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)) for c in cmds]
    failed = []
    for c, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if p.returncode != 0:
            failed.append((c, text))
        elif text:
            sys.stderr.write(text + "\n")
    if failed:
        msg = "\n\n".join(" ".join(c) + "\n" + t for c, t in failed)
        raise RuntimeError("native build failed:\n" + msg)


def build(force: bool = False, verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cmds, objs = [], []
    for s in HIP_SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(OBJ, s + ".o")
        objs.append(obj)
        if _stale(obj, src, force):
            cmds.append([HIPCC] + HIP_FLAGS + ["-c", src, "-o", obj])
    for s in CPP_SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(OBJ, s + ".o")
        objs.append(obj)
        if _stale(obj, src, force):
            cmds.append(["g++"] + CXX_FLAGS + ["-c", src, "-o", obj])
    if verbose:
        for c in cmds:
            print(" ".join(c))
    _run_all(cmds)
    if force or cmds or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        _run_all([[HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-pthread"]])
        os.replace(tmp, LIB)
    return LIB


def build_tsan(force: bool = False) -> str:
    """Scheduler core + fake backend + a C++ stress driver, built with
    -fsanitize=thread by g++ (host code only; no device code involved)."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in ("sched.cpp", "layout.cpp", "backend_fake.cpp", "tsan_main.cpp")]
    if not force and os.path.exists(TSAN_BIN) and os.path.getmtime(TSAN_BIN) >= max(
            max(os.path.getmtime(s) for s in srcs), _deps_mtime()):
        return TSAN_BIN
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-DSET_NO_HIP_BACKEND", "-I" + INCLUDE,
           "-I" + CSRC, "-pthread", "-o", TSAN_BIN] + srcs
    _run_all([cmd])
    return TSAN_BIN


TSAN_HIP_BIN = os.path.join(OBJ, "hip_backend_tsan_test")
STUB = os.path.join(CSRC, "hipstub")


def build_tsan_hip(force: bool = False) -> str:
    """The HIP backend's host code (backend_hip.hip compiled as C++) with the
    scheduler core, over the host-only runtime stand-in in csrc/hipstub, and a
    stress driver, built with -fsanitize=thread by g++ (no device code)."""
    os.makedirs(OBJ, exist_ok=True)
    hip_src = os.path.join(CSRC, "backend_hip.hip")
    srcs = [os.path.join(STUB, "hip_stub.cpp"), os.path.join(STUB, "tsan_hip_main.cpp")] + [
        os.path.join(CSRC, s) for s in ("sched.cpp", "layout.cpp", "backend_fake.cpp")]
    deps = srcs + [hip_src, os.path.join(STUB, "hip", "hip_runtime.h")]
    if not force and os.path.exists(TSAN_HIP_BIN) and os.path.getmtime(TSAN_HIP_BIN) >= max(
            max(os.path.getmtime(s) for s in deps), _deps_mtime()):
        return TSAN_HIP_BIN
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-I" + STUB, "-I" + INCLUDE, "-I" + CSRC,
           "-pthread", "-Wno-unused-function", "-o", TSAN_HIP_BIN, "-x", "c++", hip_src, "-x", "none"] + srcs
    _run_all([cmd])
    return TSAN_HIP_BIN


if __name__ == "__main__":
    force = "--force" in sys.argv
    print(build(force=force, verbose=True))
    if "--tsan" in sys.argv:
        print(build_tsan(force=force))
        print(build_tsan_hip(force=force))
