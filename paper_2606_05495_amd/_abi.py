"""ctypes binding of include/set.h: same names, argument marshalling only.

Every step of a job runs in the native library (libset.so); importing this
module fails loudly if the library has not been built.  torch is imported
first so that the library binds to the same HIP runtime torch uses (one
runtime per process: streams and device memory from torch are valid in it).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # bind to torch's HIP runtime when torch is present
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libset.so")

SET_ABI_VERSION = 4

# status codes
SET_OK, SET_EINVAL, SET_ENOMEM, SET_EDEVICE, SET_EAGAIN, SET_ETIMEOUT, SET_ECLOSED, SET_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
# modes
SET_MODE_SET, SET_MODE_SYNC, SET_MODE_GRAPH, SET_MODE_BATCH_SYNC, SET_MODE_QUEUE = 0, 1, 2, 3, 4
SET_BACKEND_HIP, SET_BACKEND_FAKE = 0, 1
SET_CB_EVENT_POLL, SET_CB_EVENT_CHAIN, SET_CB_SAME_STREAM, SET_CB_HOST_FLAG, SET_CB_EVENT_BLOCKING = 0, 1, 2, 3, 4
SET_SUBMIT_ROUND_ROBIN, SET_SUBMIT_SHORTEST, SET_SUBMIT_SKEW0 = 0, 1, 2
SET_STEAL_ANY, SET_STEAL_BUSY = 0, 1
# pipelines
SET_PIPE_BOX_HIST_U8, SET_PIPE_GAUSS_SOBEL_F32, SET_PIPE_SAXPY_TANH_SUM_F32, SET_PIPE_SCAN_I32_I64 = 0, 1, 2, 3
SET_PIPE_SAXPY_BATCH_F32 = 4
SET_PIPE_SCAN_LIB_I32_I64 = 5
SET_PIPE_HOTSPOT_F32 = 6
SET_TF_DEBUG, SET_TF_SCAN_LOW32, SET_TF_CAPTURE, SET_TF_POISON = 0x1, 0x2, 0x4, 0x8
SET_COPY_KERNELS, SET_COPY_NODES, SET_COPY_ASYNC_IN = 0, 1, 2
COPY_MODES = {"nodes": SET_COPY_NODES, "kernels": SET_COPY_KERNELS, "async_in": SET_COPY_ASYNC_IN}
SET_NONBLOCK = 0x1
SET_STAGE_INPUT_COPY, SET_STAGE_OUTPUT_COPY = -1, -2
SET_OUT_MAGIC = 0x5E7D0A11

MODES = {"set": SET_MODE_SET, "sync": SET_MODE_SYNC, "graph": SET_MODE_GRAPH, "batch": SET_MODE_BATCH_SYNC,
         "queue": SET_MODE_QUEUE}
CALLBACKS = {"event_chain": SET_CB_EVENT_CHAIN, "same_stream": SET_CB_SAME_STREAM, "event_poll": SET_CB_EVENT_POLL,
             "host_flag": SET_CB_HOST_FLAG, "event_blocking": SET_CB_EVENT_BLOCKING}


class set_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("mode", ctypes.c_int32),
        ("backend", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("num_workers", ctypes.c_int32),
        ("slots_per_worker", ctypes.c_int32),
        ("queue_capacity", ctypes.c_int32),
        ("inflight_per_worker", ctypes.c_int32),
        ("work_stealing", ctypes.c_int32),
        ("batch_size", ctypes.c_int32),
        ("callback_mode", ctypes.c_int32),
        ("submit_policy", ctypes.c_int32),
        ("spin_us", ctypes.c_int32),
        ("staging_capacity", ctypes.c_int32),
        ("mem_budget_bytes", ctypes.c_uint64),
        ("streams", ctypes.POINTER(ctypes.c_void_p)),
        ("seed", ctypes.c_uint64),
        ("fake_fail_after", ctypes.c_int32),
        ("fake_reorder_callbacks", ctypes.c_int32),
        ("dispatch_threads", ctypes.c_int32),
        ("input_copy_streams", ctypes.c_int32),
        ("callback_streams", ctypes.c_int32),
        ("steal_policy", ctypes.c_int32),
    ]


class set_job_template(ctypes.Structure):
    _fields_ = [
        ("pipeline", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("width", ctypes.c_uint32),
        ("height", ctypes.c_uint32),
        ("max_n", ctypes.c_uint64),
        ("threshold", ctypes.c_float),
        ("copy_mode", ctypes.c_uint32),
        ("arena", ctypes.c_void_p),
        ("arena_bytes", ctypes.c_uint64),
        ("dev_x_pool", ctypes.c_void_p),
        ("dev_y_pool", ctypes.c_void_p),
        ("pool_len", ctypes.c_uint64),
        ("block", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("batch_max", ctypes.c_uint32),
        ("tiles_max", ctypes.c_uint32),
        ("stress_delay_us", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class set_job_args(ctypes.Structure):
    _fields_ = [
        ("host_in", ctypes.c_void_p),
        ("in_bytes", ctypes.c_uint64),
        ("host_out", ctypes.c_void_p),
        ("out_bytes", ctypes.c_uint64),
        ("n", ctypes.c_uint64),
        ("a", ctypes.c_float),
        ("worker_hint", ctypes.c_int32),
        ("x_off", ctypes.c_uint64),
        ("y_off", ctypes.c_uint64),
        ("user_tag", ctypes.c_uint64),
        ("grid", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


# numpy mirror of set_job_args for bulk submission
JOB_ARGS_DTYPE = np.dtype({
    "names": ["host_in", "in_bytes", "host_out", "out_bytes", "n", "a", "worker_hint", "x_off", "y_off", "user_tag",
              "grid", "reserved"],
    "formats": [np.uint64, np.uint64, np.uint64, np.uint64, np.uint64, np.float32, np.int32, np.uint64, np.uint64,
                np.uint64, np.uint32, np.uint32],
    "offsets": [0, 8, 16, 24, 32, 40, 44, 48, 56, 64, 72, 76],
    "itemsize": 80,
})

# numpy mirror of set_vec_job
VEC_JOB_DTYPE = np.dtype({"names": ["x_off", "y_off", "n", "a", "reserved"],
                          "formats": [np.uint64, np.uint64, np.uint64, np.float32, np.uint32],
                          "offsets": [0, 8, 16, 24, 28], "itemsize": 32})


class set_vec_tuning(ctypes.Structure):
    _fields_ = [("tile_elems", ctypes.c_uint32 * 64), ("grid", ctypes.c_uint32 * 64)]


class set_out_header(ctypes.Structure):
    _fields_ = [
        ("job_id", ctypes.c_uint64),
        ("seq", ctypes.c_uint64),
        ("worker", ctypes.c_uint32),
        ("slot", ctypes.c_uint32),
        ("magic", ctypes.c_uint32),
        ("canary_ok", ctypes.c_uint32),
        ("user_tag", ctypes.c_uint64),
        ("reserved", ctypes.c_uint64 * 3),
    ]


OUT_HEADER_DTYPE = np.dtype([("job_id", np.uint64), ("seq", np.uint64), ("worker", np.uint32), ("slot", np.uint32),
                             ("magic", np.uint32), ("canary_ok", np.uint32), ("user_tag", np.uint64),
                             ("reserved", np.uint64, (3,))])
OUT_HEADER_BYTES = 64


class set_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("stolen", ctypes.c_uint64),
        ("failed", ctypes.c_uint64),
        ("launches_per_worker", ctypes.c_uint64 * 64),
        ("host_ns_bind", ctypes.c_uint64),
        ("host_ns_launch", ctypes.c_uint64),
        ("host_ns_callback", ctypes.c_uint64),
        ("host_ns_sync", ctypes.c_uint64),
        ("queue_high_water", ctypes.c_uint32),
        ("inflight_high_water", ctypes.c_uint32),
        ("bytes_h2d", ctypes.c_uint64),
        ("bytes_d2h", ctypes.c_uint64),
        ("mem_in_use", ctypes.c_uint64),
        ("mem_high_water", ctypes.c_uint64),
        ("batches", ctypes.c_uint64),
        ("t_first_submit_ns", ctypes.c_uint64),
        ("t_last_done_ns", ctypes.c_uint64),
    ]


JOB_TIMES_DTYPE = np.dtype([("job_id", np.uint64), ("t_submit", np.uint64), ("t_launch", np.uint64),
                            ("t_done", np.uint64), ("worker", np.int32), ("slot", np.int32), ("stolen", np.int32),
                            ("status", np.int32)])

# numpy mirror of set_request (arrival, template, job args)
REQUEST_DTYPE = np.dtype({
    "names": ["t_arrival_ns", "template_id", "reserved_r", "host_in", "in_bytes", "host_out", "out_bytes", "n", "a",
              "worker_hint", "x_off", "y_off", "user_tag", "grid", "reserved"],
    "formats": [np.uint64, np.int32, np.uint32, np.uint64, np.uint64, np.uint64, np.uint64, np.uint64, np.float32,
                np.int32, np.uint64, np.uint64, np.uint64, np.uint32, np.uint32],
    "offsets": [0, 8, 12, 16, 24, 32, 40, 48, 56, 60, 64, 72, 80, 88, 92],
    "itemsize": 96,
})


class set_serve_config(ctypes.Structure):
    _fields_ = [("vec_inflight", ctypes.c_uint32), ("vec_batch_max", ctypes.c_uint32), ("window_ns", ctypes.c_uint64),
                ("tuning", ctypes.POINTER(set_vec_tuning))]


class set_serve_stats(ctypes.Structure):
    _fields_ = [("arrived", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("not_admitted", ctypes.c_uint64), ("vec_batches", ctypes.c_uint64), ("t_start_ns", ctypes.c_uint64),
                ("t_end_ns", ctypes.c_uint64), ("max_backlog", ctypes.c_uint64)]


set_completion_fn = ctypes.CFUNCTYPE(None, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p)

# every entry point the header declares (checked by the export test)
EXPORTS = [
    "set_ctx_create", "set_ctx_destroy", "set_template_footprint", "set_template_define", "set_submit",
    "set_submit_many", "set_set_completion_cb", "set_drain", "set_get_stats", "set_reset_stats",
    "set_get_job_times", "set_time_stage", "set_time_device_copy", "set_stage_info", "set_last_error", "set_strerror",
    "set_run_vector_jobs", "set_serve", "set_job_io_bytes", "set_run_vector_jobs_noalloc",
]
SET_NOALLOC_MAX_JOBS = 16384
SET_NOALLOC_MAX_ITEMS = 1 << 20

_lib = None


def load():
    """Load libset.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("native library %s is missing: build it with `python -m paper_2606_05495_amd.build`"
                           % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    U64 = ctypes.c_uint64
    proto = {
        "set_ctx_create": (I, [ctypes.POINTER(set_config), ctypes.POINTER(P)]),
        "set_ctx_destroy": (I, [P]),
        "set_template_footprint": (I, [ctypes.POINTER(set_config), ctypes.POINTER(set_job_template),
                                       ctypes.POINTER(U64), ctypes.POINTER(U64)]),
        "set_template_define": (I, [P, ctypes.POINTER(set_job_template), ctypes.POINTER(I)]),
        "set_submit": (I, [P, I, ctypes.POINTER(set_job_args), I, ctypes.POINTER(U64)]),
        "set_submit_many": (I, [P, I, P, U64, I, ctypes.POINTER(U64)]),
        "set_set_completion_cb": (I, [P, set_completion_fn, P]),
        "set_drain": (I, [P, ctypes.c_int64]),
        "set_get_stats": (I, [P, ctypes.POINTER(set_stats)]),
        "set_reset_stats": (I, [P]),
        "set_get_job_times": (I, [P, P, U64, ctypes.POINTER(U64)]),
        "set_time_stage": (I, [P, I, I, I, I, ctypes.POINTER(ctypes.c_double)]),
        "set_time_device_copy": (I, [P, U64, I, ctypes.POINTER(ctypes.c_double)]),
        "set_stage_info": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(U64), I, ctypes.c_char_p, I]),
        "set_job_io_bytes": (I, [P, I, U64, ctypes.POINTER(U64), ctypes.POINTER(U64)]),
        "set_run_vector_jobs": (I, [P, I, P, U64, P, ctypes.POINTER(set_vec_tuning), ctypes.POINTER(U64)]),
        "set_serve": (I, [P, P, U64, ctypes.POINTER(set_serve_config), P, P, ctypes.POINTER(set_serve_stats)]),
        "set_run_vector_jobs_noalloc": (I, [I, P, P, P, U64, U64, P, U64, P, ctypes.POINTER(set_vec_tuning),
                                            ctypes.c_uint32]),
        "set_last_error": (ctypes.c_char_p, [P]),
        "set_strerror": (ctypes.c_char_p, [I]),
    }
    for name, (res, args) in proto.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class SetError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (load().set_strerror(code).decode(), msg))
        self.code = code


def check(rc, ctx=None):
    if rc != SET_OK:
        msg = load().set_last_error(ctx).decode(errors="replace")
        raise SetError(rc, msg)
    return rc


# ------------------------------------------------------------------ same-name wrappers
def set_ctx_create(cfg: set_config):
    h = ctypes.c_void_p()
    check(load().set_ctx_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def set_ctx_destroy(ctx):
    return load().set_ctx_destroy(ctx)


def set_template_footprint(cfg, tmpl):
    s, t = ctypes.c_uint64(), ctypes.c_uint64()
    check(load().set_template_footprint(ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(tmpl),
                                        ctypes.byref(s), ctypes.byref(t) if cfg is not None else None))
    return s.value, t.value


def set_template_define(ctx, tmpl: set_job_template) -> int:
    tid = ctypes.c_int()
    check(load().set_template_define(ctx, ctypes.byref(tmpl), ctypes.byref(tid)), ctx)
    return tid.value


def set_submit(ctx, template_id: int, args: set_job_args, flags: int = 0) -> int:
    jid = ctypes.c_uint64()
    rc = load().set_submit(ctx, template_id, ctypes.byref(args), flags, ctypes.byref(jid))
    if rc == SET_EAGAIN:
        return -1
    check(rc, ctx)
    return jid.value


def set_submit_many(ctx, template_id: int, args: np.ndarray, flags: int = 0) -> int:
    assert args.dtype == JOB_ARGS_DTYPE and args.flags["C_CONTIGUOUS"]
    first = ctypes.c_uint64()
    check(load().set_submit_many(ctx, template_id, args.ctypes.data, args.size, flags, ctypes.byref(first)), ctx)
    return first.value


def set_set_completion_cb(ctx, fn, user=None):
    check(load().set_set_completion_cb(ctx, fn if fn is not None else set_completion_fn(0), user), ctx)


def set_drain(ctx, timeout_ns: int = -1):
    return check(load().set_drain(ctx, timeout_ns), ctx)


def set_get_stats(ctx) -> set_stats:
    st = set_stats()
    check(load().set_get_stats(ctx, ctypes.byref(st)), ctx)
    return st


def set_reset_stats(ctx):
    check(load().set_reset_stats(ctx), ctx)


def set_get_job_times(ctx, max_records: int = 1 << 22) -> np.ndarray:
    out = np.zeros(max_records, dtype=JOB_TIMES_DTYPE)
    n = ctypes.c_uint64()
    check(load().set_get_job_times(ctx, out.ctypes.data, max_records, ctypes.byref(n)), ctx)
    return out[:n.value]


def set_time_device_copy(ctx, nbytes: int, reps: int) -> float:
    us = ctypes.c_double()
    check(load().set_time_device_copy(ctx, nbytes, reps, ctypes.byref(us)), ctx)
    return us.value


def set_time_stage(ctx, template_id: int, stage: int, worker: int, reps: int) -> float:
    us = ctypes.c_double()
    check(load().set_time_stage(ctx, template_id, stage, worker, reps, ctypes.byref(us)), ctx)
    return us.value


def set_job_io_bytes(ctx, template_id: int, n: int = 0):
    i, o = ctypes.c_uint64(), ctypes.c_uint64()
    check(load().set_job_io_bytes(ctx, template_id, n, ctypes.byref(i), ctypes.byref(o)), ctx)
    return i.value, o.value


def set_stage_info(ctx, template_id: int):
    n = ctypes.c_int()
    b = (ctypes.c_uint64 * 64)()
    names = ctypes.create_string_buffer(64 * 32)
    check(load().set_stage_info(ctx, template_id, ctypes.byref(n), b, 64, names, 64 * 32), ctx)
    return list(zip(names.value.decode().split(","), list(b)[:n.value]))


def set_run_vector_jobs(ctx, template_id: int, jobs: np.ndarray, results: np.ndarray, tuning=None) -> int:
    assert jobs.dtype == VEC_JOB_DTYPE and jobs.flags["C_CONTIGUOUS"]
    assert results.dtype == np.float32 and results.size >= jobs.size and results.flags["C_CONTIGUOUS"]
    nb = ctypes.c_uint64()
    check(load().set_run_vector_jobs(ctx, template_id, jobs.ctypes.data, jobs.size, results.ctypes.data,
                                     ctypes.byref(tuning) if tuning is not None else None, ctypes.byref(nb)), ctx)
    return nb.value


def set_run_vector_jobs_noalloc(device: int, stream: int, dev_x_pool: int, dev_y_pool: int, pool_len: int,
                                max_n: int, dev_jobs: int, count: int, dev_results: int, tuning=None,
                                grid: int = 0) -> None:
    """Device pointers and the stream as integers; enqueues only (results are
    ready once the stream has reached them)."""
    check(load().set_run_vector_jobs_noalloc(device, stream, dev_x_pool, dev_y_pool, pool_len, max_n, dev_jobs,
                                             count, dev_results,
                                             ctypes.byref(tuning) if tuning is not None else None, grid))


def set_serve(ctx, reqs: np.ndarray, cfg: set_serve_config = None, vec_results: np.ndarray = None):
    """Returns (done_ns array, stats)."""
    assert reqs.dtype == REQUEST_DTYPE and reqs.flags["C_CONTIGUOUS"]
    done = np.zeros(reqs.size, np.uint64)
    st = set_serve_stats()
    vr = vec_results.ctypes.data if vec_results is not None else None
    check(load().set_serve(ctx, reqs.ctypes.data, reqs.size, ctypes.byref(cfg) if cfg is not None else None,
                           done.ctypes.data, vr, ctypes.byref(st)), ctx)
    return done, st


def set_last_error(ctx) -> str:
    return load().set_last_error(ctx).decode(errors="replace")


def set_strerror(code: int) -> str:
    return load().set_strerror(code).decode()
