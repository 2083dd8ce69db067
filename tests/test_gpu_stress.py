"""Memory-safety stress on the GPU: the rule that no job writes into a slot
another job still uses (paper Section 4.1), under Algorithms 1-3's release
and stealing.

Templates with the poison option end every job's graph, after its output
copy, with a kernel that fills the slot's buffers with 0xFF bytes (and fill
them once when defined); the delay option puts a kernel that waits before
every job's first stage, widening the window in which a slot released too
early would be overwritten by the next job's input copy.  Under skewed
submission (every job to worker 0, so the other workers steal), each result
must match the oracle, carry its own job id and tag and report intact
canaries, and the runs with one slot per worker and with sixteen must give
bit-identical outputs.
"""
import numpy as np
import pytest

import oracle
from paper_2606_05495_amd import _abi as A
from paper_2606_05495_amd import synth
from paper_2606_05495_amd.runtime import Context, out_header, pinned

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _up64(v):
    return (v + 63) // 64 * 64


def _ctx(mode, slots, callback="event_poll", copy_streams=0, workers=4):
    return Context(mode=mode, workers=workers, slots=slots, callback=callback,
                   submit_policy=A.SET_SUBMIT_SKEW0 if mode == "set" else A.SET_SUBMIT_ROUND_ROBIN,
                   dispatchers=2 if mode == "set" else 1, input_copy_streams=copy_streams)


def _submit(ctx, tid, inputs, ob):
    """Submit one job per input (bytes), wait, return (outputs, first id, stats)."""
    k = len(inputs)
    istride = _up64(max(len(v) for v in inputs))
    ostride = _up64(max(ob))
    tin, nin = pinned(istride * k)
    tout, nout = pinned(ostride * k)
    arr = ctx.job_array(k)
    for i, v in enumerate(inputs):
        nin[i * istride:i * istride + len(v)] = v
        arr[i]["host_in"] = tin.data_ptr() + i * istride
        arr[i]["in_bytes"] = len(v)
        arr[i]["host_out"] = tout.data_ptr() + i * ostride
        arr[i]["out_bytes"] = ob[i]
        arr[i]["user_tag"] = 7000 + i
    first = ctx.submit_many(tid, arr)
    ctx.drain()
    st = ctx.stats()
    outs = []
    for i in range(k):
        o = nout[i * ostride:i * ostride + ob[i]].copy()
        h = out_header(o)
        assert h["magic"] == A.SET_OUT_MAGIC and h["canary_ok"] == 1, (i, h)
        assert h["job_id"] == first + i and h["user_tag"] == 7000 + i, (i, h)
        outs.append(o)
    return outs, first, st


# ------------------------------------------------------------------ Gaussian / Sobel, every mode, d = 1 vs d = 16
IMG_H, IMG_W, IMG_JOBS = 256, 256, 48
STRESS = [("set", "event_poll", "kernels", 0), ("set", "event_poll", "async_in", 2),
          ("set", "event_chain", "nodes", 0), ("set", "host_flag", "kernels", 0),
          ("set", "event_blocking", "async_in", 2), ("queue", "event_poll", "kernels", 0),
          ("batch", "event_poll", "async_in", 0), ("sync", "event_poll", "kernels", 0),
          ("graph", "event_poll", "nodes", 0)]


def _gauss_run(mode, slots, callback, copy, copy_streams, imgs, capture=False):
    ctx = _ctx(mode, slots, callback, copy_streams)
    flags = A.SET_TF_POISON | A.SET_TF_DEBUG | (A.SET_TF_CAPTURE if capture else 0)
    tid = ctx.define("gauss_sobel", width=IMG_W, height=IMG_H, flags=flags, copy=copy, stress_delay_us=50)
    ob = ctx.out_bytes(tid)
    outs, _, st = _submit(ctx, tid, [im.ravel().view(np.uint8) for im in imgs], [ob] * len(imgs))
    ctx.close()
    return outs, st


def _check_gauss(img, o):
    """Per pixel: blur within 1e-5 of the convolution of |input|, mask exact
    outside the threshold band, count within the band, sum within 1e-5."""
    h, w = img.shape
    ref = oracle.gauss_sobel(img)
    absconv = oracle.gauss_sobel(np.abs(img))["blur"]
    b_off = _up64(128 + h * w)
    blur = o[b_off:b_off + 4 * h * w].view(np.float32).reshape(h, w)
    assert np.all(np.abs(blur.astype(np.float64) - ref["blur"]) <= 1e-5 * absconv + 1e-30)
    mask = o[128:128 + h * w].reshape(h, w)
    outside = np.abs(ref["mag"] - 1.0) > oracle.BAND_EPS
    assert np.array_equal(mask[outside], ref["mask"][outside])
    count = int(o[64:68].view(np.uint32)[0])
    s = float(o[68:72].view(np.float32)[0])
    assert abs(count - ref["count"]) <= ref["band"]
    assert abs(s - ref["sum"]) <= 1e-5 * abs(ref["sum"]) + 1e-6


@pytest.fixture(scope="module")
def stress_images():
    return [synth.normal_image(11, k, IMG_H, IMG_W) for k in range(IMG_JOBS)]


@pytest.mark.parametrize("mode,callback,copy,copy_streams", STRESS)
def test_poison_and_delay_one_vs_sixteen_slots(torch_gpu, stress_images, mode, callback, copy, copy_streams):
    _say("stress", mode, callback, copy, copy_streams)
    imgs = stress_images
    o1, st1 = _gauss_run(mode, 1, callback, copy, copy_streams, imgs)
    o16, st16 = _gauss_run(mode, 16, callback, copy, copy_streams, imgs)
    for img, a in zip(imgs, o1):
        _check_gauss(img, a)
    for a, b in zip(o1, o16):  # payloads bit-identical (the headers differ in worker / slot / id)
        assert np.array_equal(a[64:], b[64:])
    assert st1.completed == st16.completed == IMG_JOBS
    if mode == "set":
        assert st1.stolen > 0 and st16.stolen > 0, (st1.stolen, st16.stolen)


def test_poison_with_captured_templates(torch_gpu, stress_images):
    """The capture path places the delay and poison kernels in the chain too."""
    _say("stress captured")
    imgs = stress_images[:16]
    o, st = _gauss_run("set", 2, "event_poll", "kernels", 0, imgs, capture=True)
    for img, a in zip(imgs, o):
        _check_gauss(img, a)
    assert st.stolen > 0


# ------------------------------------------------------------------ what the poison leaves in the slots
def test_poison_fills_every_slot_after_each_job(torch_gpu):
    """Slot layout: a 256-byte header block, the buffers, a 256-byte tail
    canary block.  After the jobs (and right after the template is defined)
    every byte between the header block and the tail block is 0xFF, while the
    canaries and the last job's header stay."""
    _say("poison contents")
    ctx = Context(mode="set", workers=2, slots=3)
    h, w = 70, 100
    tid = ctx.define("gauss_sobel", width=w, height=h, flags=A.SET_TF_POISON, copy="kernels")
    slot_bytes, total = A.set_template_footprint(ctx.cfg, ctx.templates[tid])
    nslots = 6
    torch_gpu.cuda.synchronize()
    arena0 = ctx.arenas[tid][:total].cpu().numpy()
    for k in range(nslots):
        s = arena0[k * slot_bytes:(k + 1) * slot_bytes]
        assert np.all(s[256:slot_bytes - 256] == 0xFF), k
    imgs = [synth.normal_image(5, k, h, w) for k in range(12)]
    outs, first, _ = _submit(ctx, tid, [im.ravel().view(np.uint8) for im in imgs], [ctx.out_bytes(tid)] * 12)
    for img, o in zip(imgs, outs):
        ref = oracle.gauss_sobel(img, want_images=False)
        assert abs(int(o[64:68].view(np.uint32)[0]) - ref["count"]) <= ref["band"]
    torch_gpu.cuda.synchronize()
    arena = ctx.arenas[tid][:total].cpu().numpy()
    last_ids = {}
    for i, o in enumerate(outs):
        hd = out_header(o)
        last_ids[(int(hd["worker"]), int(hd["slot"]))] = first + i
    for k in range(nslots):
        s = arena[k * slot_bytes:(k + 1) * slot_bytes]
        assert np.all(s[256:slot_bytes - 256] == 0xFF), k
        assert np.array_equal(s[:8], arena0[k * slot_bytes:k * slot_bytes + 8])  # head canary
        assert np.array_equal(s[slot_bytes - 256:slot_bytes - 248],
                              arena0[(k + 1) * slot_bytes - 256:(k + 1) * slot_bytes - 248])  # tail canary
        wk, sk = divmod(k, 3)
        if (wk, sk) in last_ids:  # the header keeps the id of the slot's last job
            assert int(s[8:16].view(np.uint64)[0]) == last_ids[(wk, sk)]
    ctx.close()


# ------------------------------------------------------------------ other pipelines under poison
def test_poison_scan_ragged_tails(torch_gpu):
    """The scan reads its ragged last tile in whole 8-value groups and zeroes
    what lies past n; with the slot's padding poisoned (0xFF = -1 per int32)
    instead of zero-filled, the sums must still be exact."""
    _say("poison scan")
    rng = np.random.default_rng(21)
    ns = [1, 7, 9, 2047, 2049, 100003, 1 << 17, 5, 131071]
    inputs = [rng.integers(-(1 << 20), (1 << 20) + 1, n).astype(np.int32) for n in ns]
    ctx = _ctx("set", 1)
    tid = ctx.define("scan", max_n=1 << 17, flags=A.SET_TF_POISON, copy="kernels", stress_delay_us=20)
    ob = [ctx.out_bytes(tid, len(v)) for v in inputs]
    jobs = [v.view(np.uint8) for v in inputs]
    k = len(jobs)
    tin, nin = pinned(sum(_up64(len(v)) for v in jobs))
    tout, nout = pinned(sum(_up64(b) for b in ob))
    arr = ctx.job_array(k)
    oi = oo = 0
    offs = []
    for i, v in enumerate(jobs):
        nin[oi:oi + len(v)] = v
        arr[i]["host_in"] = tin.data_ptr() + oi
        arr[i]["in_bytes"] = len(v)
        arr[i]["host_out"] = tout.data_ptr() + oo
        arr[i]["out_bytes"] = ob[i]
        arr[i]["n"] = len(inputs[i])
        offs.append(oo)
        oi += _up64(len(v))
        oo += _up64(ob[i])
    first = ctx.submit_many(tid, arr)
    ctx.drain()
    for i, v in enumerate(inputs):
        o = nout[offs[i]:offs[i] + ob[i]]
        hd = out_header(o)
        assert hd["magic"] == A.SET_OUT_MAGIC and hd["canary_ok"] == 1 and hd["job_id"] == first + i
        assert np.array_equal(o[64:].view(np.int64), oracle.scan(v)), ns[i]
    ctx.close()


def test_poison_library_scan_template(torch_gpu):
    """The captured library call (rocPRIM's scan between the bracket kernels)
    with poisoned slots: bit-exact sums, job after job in the same slots."""
    _say("poison library scan")
    n = 100003
    rng = np.random.default_rng(22)
    inputs = [rng.integers(-(1 << 20), (1 << 20) + 1, n).astype(np.int32) for _ in range(6)]
    ctx = _ctx("set", 1, workers=2)
    tid = ctx.define("scan_lib", max_n=n, flags=A.SET_TF_POISON, copy="kernels", stress_delay_us=20)
    ob = ctx.out_bytes(tid, n)
    outs, _, _ = _submit(ctx, tid, [v.view(np.uint8) for v in inputs], [ob] * len(inputs))
    for v, o in zip(inputs, outs):
        assert np.array_equal(o[64:64 + 8 * n].view(np.int64), oracle.scan(v))
    ctx.close()


def test_poison_thermal_grid(torch_gpu):
    """Every step reads the previous step's buffer: none may see poison."""
    _say("poison hotspot")
    h, w = 97, 130
    grids = [synth.hotspot_input(3, k, h, w) for k in range(8)]
    ctx = _ctx("set", 1)
    tid = ctx.define("hotspot", width=w, height=h, max_n=5, flags=A.SET_TF_POISON, copy="async_in",
                     stress_delay_us=20)
    ob = ctx.out_bytes(tid)
    inputs = [np.concatenate([t0.ravel(), p.ravel()]).astype(np.float32).view(np.uint8) for t0, p in grids]
    outs, _, _ = _submit(ctx, tid, inputs, [ob] * len(grids))
    for (t0, p), o in zip(grids, outs):
        ref = oracle.hotspot(t0, p, 5)
        got = o[64:64 + 4 * h * w].view(np.float32).reshape(h, w)
        assert np.max(np.abs(got - ref)) <= oracle.hotspot_tolerance(ref, 5)
    ctx.close()


def test_poison_keeps_the_batch_work_counter(torch_gpu):
    """Batched vector templates carry one word from batch to batch (the work
    counter, rewound by each batch's last stage); the poison kernel writes it
    as zero, so results match those of a template without poison, bit for
    bit, batch after batch."""
    _say("poison vector batches")
    L = 1 << 23
    x = synth.vec_pool(0, "x", L)
    y = synth.vec_pool(0, "y", L)
    xd = torch_gpu.from_numpy(x).cuda()
    yd = torch_gpu.from_numpy(y).cuda()
    js = synth.vec_jobs(4, 200, pool_len=L)
    jobs = np.zeros(200, dtype=A.VEC_JOB_DTYPE)
    for f in ("n", "a", "x_off", "y_off"):
        jobs[f] = js[f]
    res = {}
    for poison in (False, True):
        ctx = Context(mode="set", workers=4, slots=2)
        tid = ctx.define("saxpy_batch", max_n=1 << 22, x_pool=xd, y_pool=yd, batch_max=16, tiles_max=1024,
                         flags=A.SET_TF_POISON if poison else 0)
        r1, _ = ctx.run_vector_jobs(tid, jobs)
        r2, _ = ctx.run_vector_jobs(tid, jobs)
        assert np.array_equal(r1.view(np.uint32), r2.view(np.uint32))
        res[poison] = r1
        if poison:
            slot_bytes, total = A.set_template_footprint(ctx.cfg, ctx.templates[tid])
            torch_gpu.cuda.synchronize()
            arena = ctx.arenas[tid][:total].cpu().numpy()
            for k in range(8):
                body = arena[k * slot_bytes + 256:(k + 1) * slot_bytes - 256].view(np.uint32)
                assert int(np.count_nonzero(body != 0xFFFFFFFF)) == 1 and int(np.count_nonzero(body == 0)) == 1
        ctx.close()
    assert np.array_equal(res[False].view(np.uint32), res[True].view(np.uint32))
    for i in range(0, 200, 20):
        n, xo, yo = int(jobs["n"][i]), int(jobs["x_off"][i]), int(jobs["y_off"][i])
        S, E = oracle.saxpy_tanh_sum(x[xo:xo + n], y[yo:yo + n], jobs["a"][i])
        assert abs(float(res[True][i]) - S) <= oracle.vec_tolerance(S, E)
