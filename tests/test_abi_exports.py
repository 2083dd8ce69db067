"""The C-ABI library loads and exports every symbol include/set.h declares (no compute)."""
import ctypes
import os
import re

from paper_2606_05495_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "set.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(set_[a-z_]+)\s*\(", text, re.M)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(A.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = A.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(A.set_config) == 104
    assert ctypes.sizeof(A.set_job_args) == 80 == A.JOB_ARGS_DTYPE.itemsize
    assert ctypes.sizeof(A.set_out_header) == 64 == A.OUT_HEADER_DTYPE.itemsize
    assert ctypes.sizeof(A.set_job_template) == 96
    assert A.VEC_JOB_DTYPE.itemsize == 32 and ctypes.sizeof(A.set_vec_tuning) == 512
    assert A.REQUEST_DTYPE.itemsize == 96 and ctypes.sizeof(A.set_serve_config) == 24
    for f, off in (("a", 40), ("worker_hint", 44), ("x_off", 48), ("user_tag", 64)):
        assert getattr(A.set_job_args, f).offset == off


def test_strerror_and_create_errors():
    assert A.set_strerror(A.SET_EDEVICE) == "SET_EDEVICE"
    cfg = A.set_config()
    cfg.abi_version = 999
    h = ctypes.c_void_p()
    rc = A.load().set_ctx_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == A.SET_EINVAL and not h.value
    assert "abi_version" in A.set_last_error(None)


def test_callback_streams_range():
    """callback_streams takes 0..64 and steal_policy SET_STEAL_ANY or
    SET_STEAL_BUSY (checked before any device is touched: the fake backend
    serves here)."""
    def create(**fields):
        cfg = A.set_config()
        cfg.abi_version = A.SET_ABI_VERSION
        cfg.backend = A.SET_BACKEND_FAKE
        cfg.num_workers, cfg.slots_per_worker = 4, 2
        cfg.callback_mode = A.SET_CB_EVENT_CHAIN
        for k, v in fields.items():
            setattr(cfg, k, v)
        h = ctypes.c_void_p()
        rc = A.load().set_ctx_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc == A.SET_OK:
            A.load().set_ctx_destroy(h)
        return rc
    for k in (0, 1, 4, 64):
        assert create(callback_streams=k) == A.SET_OK
    for k in (-1, 65):
        assert create(callback_streams=k) == A.SET_EINVAL
    for p in (A.SET_STEAL_ANY, A.SET_STEAL_BUSY):
        assert create(steal_policy=p) == A.SET_OK
    for p in (-1, 2):
        assert create(steal_policy=p) == A.SET_EINVAL


def test_footprint_is_host_only():
    cfg = A.set_config()
    cfg.abi_version = A.SET_ABI_VERSION
    cfg.num_workers, cfg.slots_per_worker = 8, 16
    t = A.set_job_template()
    t.pipeline = A.SET_PIPE_GAUSS_SOBEL_F32
    t.width = t.height = 1024
    slot, total = A.set_template_footprint(cfg, t)
    # input 4 MiB + blur 4 MiB + mask 1 MiB + small
    assert 9 * 2 ** 20 <= slot < 9 * 2 ** 20 + 64 * 1024
    assert total == 128 * slot


def test_noalloc_limits_refused_on_the_host():
    """The no-allocation call checks its limits before touching a device, so
    these run without a GPU."""
    lib = A.load()
    big = A.SET_NOALLOC_MAX_JOBS + 1
    assert lib.set_run_vector_jobs_noalloc(0, None, 16, 16, 1 << 20, 4096, 16, big, 16, None, 0) == A.SET_EINVAL
    assert "16384" in A.set_last_error(None)
    # 16384 jobs of up to 2^22 elements in 1024-element items need far more than 2^20 items
    t = A.set_vec_tuning()
    for b in range(64):
        t.tile_elems[b] = 1024
    assert lib.set_run_vector_jobs_noalloc(0, None, 16, 16, 1 << 23, 1 << 22, 16, 16384, 16, ctypes.byref(t),
                                           0) == A.SET_EINVAL
    assert "work items" in A.set_last_error(None)
    t.tile_elems[5] = 1000
    assert lib.set_run_vector_jobs_noalloc(0, None, 16, 16, 1 << 23, 1 << 22, 16, 1, 16, ctypes.byref(t),
                                           0) == A.SET_EINVAL
    assert lib.set_run_vector_jobs_noalloc(0, None, None, 16, 1 << 23, 4096, 16, 1, 16, None, 0) == A.SET_EINVAL
    assert lib.set_run_vector_jobs_noalloc(0, None, 16, 16, 1 << 23, 0, 16, 1, 16, None, 0) == A.SET_EINVAL


def test_image_and_grid_size_limits():
    """Widths up to 2^20, heights up to 2^19 (so that no launch grid passes
    65,536 blocks in its second dimension) and at most 2^28 pixels, checked
    on the host."""
    cfg = A.set_config()
    cfg.abi_version = A.SET_ABI_VERSION
    cfg.num_workers, cfg.slots_per_worker = 1, 1

    def fits(pipeline, w, h):
        t = A.set_job_template()
        t.pipeline = pipeline
        t.width, t.height = w, h
        if pipeline == A.SET_PIPE_HOTSPOT_F32:
            t.max_n = 2
        try:
            A.set_template_footprint(cfg, t)
            return True
        except A.SetError as e:
            assert e.code == A.SET_EINVAL
            return False
    for p in (A.SET_PIPE_GAUSS_SOBEL_F32, A.SET_PIPE_BOX_HIST_U8, A.SET_PIPE_HOTSPOT_F32):
        assert fits(p, 4, 1 << 19) and fits(p, 1 << 20, 256) and fits(p, 512, 1 << 19)
        assert not fits(p, 4, (1 << 19) + 1)
        assert not fits(p, (1 << 20) + 1, 1)
        assert not fits(p, 1024, 1 << 19)  # 2^29 pixels
