"""Thin convenience layer over the C ABI.

PyTorch supplies plumbing only: the worker streams, each template's device
arena, the device-resident vector pools and pinned host buffers.  All job work
(copies, kernels, scheduling) happens in libset.so.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi as A

PIPELINES = {
    "box_hist": A.SET_PIPE_BOX_HIST_U8,
    "gauss_sobel": A.SET_PIPE_GAUSS_SOBEL_F32,
    "saxpy_tanh_sum": A.SET_PIPE_SAXPY_TANH_SUM_F32,
    "scan": A.SET_PIPE_SCAN_I32_I64,
    "saxpy_batch": A.SET_PIPE_SAXPY_BATCH_F32,
    "scan_lib": A.SET_PIPE_SCAN_LIB_I32_I64,
    "hotspot": A.SET_PIPE_HOTSPOT_F32,
}


def _torch():
    import torch
    return torch


def pinned(nbytes: int):
    """A pinned host buffer (torch uint8 tensor) and a numpy view of it."""
    torch = _torch()
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, pin_memory=True)
    return t, t.numpy()


def host_buffer(nbytes: int, pin: bool = True):
    """Host buffer for job inputs/outputs: pinned when a GPU is used, plain otherwise."""
    if pin:
        return pinned(nbytes)
    arr = np.zeros(max(int(nbytes), 1), np.uint8)
    return arr, arr


class Context:
    """One SET context: b workers (streams), d slots each, and its templates."""

    def __init__(self, mode="set", workers=8, slots=16, backend="hip", queue_capacity=0, inflight=0,
                 stealing=True, batch_size=0, callback="event_poll", submit_policy=A.SET_SUBMIT_ROUND_ROBIN,
                 spin_us=0, staging=0, mem_budget=0, device=0, seed=0, borrow_streams=True,
                 fake_fail_after=0, fake_reorder=False, dispatchers=1, input_copy_streams=0,
                 callback_streams=0, steal_policy=0):
        self.backend = backend
        self.workers = workers
        self.slots = slots
        self._keep = []
        cfg = A.set_config()
        cfg.abi_version = A.SET_ABI_VERSION
        cfg.mode = A.MODES[mode] if isinstance(mode, str) else int(mode)
        cfg.backend = A.SET_BACKEND_HIP if backend == "hip" else A.SET_BACKEND_FAKE
        cfg.device = device
        cfg.num_workers = workers
        cfg.slots_per_worker = slots
        cfg.queue_capacity = queue_capacity
        cfg.inflight_per_worker = inflight
        cfg.work_stealing = 1 if stealing else 0
        cfg.batch_size = batch_size
        cfg.callback_mode = A.CALLBACKS[callback] if isinstance(callback, str) else int(callback)
        cfg.submit_policy = submit_policy
        cfg.spin_us = spin_us
        cfg.staging_capacity = staging
        cfg.mem_budget_bytes = mem_budget
        cfg.seed = seed
        cfg.fake_fail_after = fake_fail_after
        cfg.fake_reorder_callbacks = 1 if fake_reorder else 0
        cfg.dispatch_threads = dispatchers
        cfg.input_copy_streams = input_copy_streams
        cfg.callback_streams = callback_streams
        cfg.steal_policy = steal_policy
        self.streams = []
        if backend == "hip" and borrow_streams:
            torch = _torch()
            dev = torch.device("cuda", device)
            self.streams = [torch.cuda.Stream(device=dev) for _ in range(workers)]
            arr = (ctypes.c_void_p * workers)(*[s.cuda_stream for s in self.streams])
            self._keep.append(arr)
            cfg.streams = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        self.cfg = cfg
        self.h = A.set_ctx_create(cfg)
        self.templates = {}
        self.arenas = {}

    # ------------------------------------------------------------ templates
    def define(self, pipeline, width=0, height=0, max_n=0, flags=0, threshold=0.0, x_pool=None, y_pool=None,
               borrow_arena=True, pool_ptrs=None, copy="kernels", batch_max=0, tiles_max=0, grid=0, block=0,
               stress_delay_us=0):
        t = A.set_job_template()
        t.pipeline = PIPELINES[pipeline] if isinstance(pipeline, str) else int(pipeline)
        t.flags = flags
        t.width = width
        t.height = height
        t.max_n = max_n
        t.threshold = threshold
        t.copy_mode = A.COPY_MODES[copy] if isinstance(copy, str) else int(copy)
        t.batch_max = batch_max
        t.tiles_max = tiles_max
        t.grid = grid
        t.block = block
        t.stress_delay_us = stress_delay_us
        if x_pool is not None:
            t.dev_x_pool = x_pool.data_ptr()
            t.dev_y_pool = y_pool.data_ptr()
            t.pool_len = min(x_pool.numel(), y_pool.numel())
            self._keep += [x_pool, y_pool]
        elif pool_ptrs is not None:  # raw device addresses (x, y, length)
            t.dev_x_pool, t.dev_y_pool, t.pool_len = pool_ptrs
        slot_bytes, total = A.set_template_footprint(self.cfg, t)
        arena = None
        if self.backend == "hip" and borrow_arena:
            torch = _torch()
            arena = torch.empty(total, dtype=torch.uint8, device=torch.device("cuda", self.cfg.device))
            self._keep.append(arena)
            t.arena = arena.data_ptr()
            t.arena_bytes = total
        tid = A.set_template_define(self.h, t)
        self.templates[tid] = t
        if arena is not None:  # the device buffer that holds every slot of the template
            self.arenas[tid] = arena
        return tid

    def in_bytes(self, tid, n=0):
        """Input bytes of a job of length n (0 = the template's max_n where that applies)."""
        return A.set_job_io_bytes(self.h, tid, n)[0]

    def out_bytes(self, tid, n=0):
        """Output bytes (header + payload) of a job of length n."""
        return A.set_job_io_bytes(self.h, tid, n)[1]

    # ------------------------------------------------------------ jobs
    @staticmethod
    def job_array(count):
        a = np.zeros(count, dtype=A.JOB_ARGS_DTYPE)
        a["worker_hint"] = -1
        return a

    def submit(self, tid, host_in=0, in_bytes=0, host_out=0, out_bytes=0, n=0, a=0.0, x_off=0, y_off=0,
               user_tag=0, worker_hint=-1, flags=0):
        args = A.set_job_args(host_in, in_bytes, host_out, out_bytes, n, a, worker_hint, x_off, y_off, user_tag)
        return A.set_submit(self.h, tid, args, flags)

    def submit_many(self, tid, arr, flags=0):
        return A.set_submit_many(self.h, tid, np.ascontiguousarray(arr), flags)

    def run_vector_jobs(self, tid, jobs, results=None, tuning=None):
        """Bucketed persistent batching of vector jobs (structured array of VEC_JOB_DTYPE)."""
        jobs = np.ascontiguousarray(jobs, dtype=A.VEC_JOB_DTYPE)
        if results is None:
            results = np.zeros(jobs.size, np.float32)
        nb = A.set_run_vector_jobs(self.h, tid, jobs, results, tuning)
        return results, nb

    def drain(self, timeout_ns=-1):
        return A.set_drain(self.h, timeout_ns)

    def stats(self):
        return A.set_get_stats(self.h)

    def reset_stats(self):
        A.set_reset_stats(self.h)

    def job_times(self):
        return A.set_get_job_times(self.h)

    def time_stage(self, tid, stage, worker=0, reps=100):
        return A.set_time_stage(self.h, tid, stage, worker, reps)

    def time_device_copy(self, nbytes, reps=100):
        """Mean time of a plain device copy kernel moving nbytes (half read, half written), cold."""
        return A.set_time_device_copy(self.h, nbytes, reps)

    def stage_info(self, tid):
        return A.set_stage_info(self.h, tid)

    def close(self):
        if self.h is not None:
            A.set_ctx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def out_header(buf: np.ndarray, offset: int = 0) -> np.ndarray:
    """Parse the 64-byte set_out_header at buf[offset:]."""
    return np.frombuffer(buf, dtype=A.OUT_HEADER_DTYPE, count=1, offset=offset)[0]
