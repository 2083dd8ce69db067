#!/usr/bin/env python3
"""Benchmark of the event-chained (SET) job scheduler on one MI355X.

Workload (one "step" = one pass of the whole job path over one batch):
10,000 jobs, each H2D of a 1024x1024 float32 N(0,1) image (pinned pool of 61
images, job j uses entry j mod 61) -> separable 5x5 Gaussian (sigma 1,
replicated borders) -> Sobel magnitude -> threshold 1.0 -> uint32 count +
float32 magnitude sum -> D2H, on 8 worker streams x 16 buffer slots.

The same jobs are also run through the batch-synchronised fixed-stream graph
baseline (one graph of 8 job chains, host sync per batch), the single-stream
synchronous baseline and the queue model, on the same GPU, and through SET
with each other completion mechanism; every result is checked against the CPU
oracle after the timed regions.  Before it touches the GPU, the run traces
short child runs of SET and batch-sync with rocprofv3 for the kernel gap and
GPU-idle fraction.  The line also carries four more workloads, each verified:
64 box/histogram jobs (the plain synchronous method against SET, bit-exact),
100,000 uneven vector jobs (bucketed persistent batches and per-job graphs
against per-job baselines), 20,000 copy-bound scan jobs (SET with and
without stealing against batch-sync) and the serving loop (open-loop arrivals
at 2k, 10k and 40k requests/s, p50/p99 latency).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import concurrent.futures
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "jobs/s and mean kernel gap (µs) vs batch-sync hipGraph; p50/p99 job latency"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_jobs(ctx, tid, n_jobs, tin, pool, ib, tout, ob, stride):
    arr = ctx.job_array(n_jobs)
    j = np.arange(n_jobs, dtype=np.uint64)
    arr["host_in"] = tin.data_ptr() + (j % np.uint64(pool)) * np.uint64(ib)
    arr["in_bytes"] = ib
    arr["host_out"] = tout.data_ptr() + j * np.uint64(stride)
    arr["out_bytes"] = ob
    arr["user_tag"] = j
    return arr


def run_mode(mode, args, jobs_per_step, steps, warmup, tin, tout, pool, torch, callback="event_chain", copy=None,
             copy_streams=None, callback_streams=0):
    from paper_2606_05495_amd.runtime import Context
    workers = args.workers
    ctx = Context(mode=mode, workers=workers, slots=args.slots if mode == "set" else 1,
                  batch_size=args.batch if mode == "batch" else 0, callback=callback, inflight=args.inflight,
                  spin_us=args.spin_us, dispatchers=args.dispatchers,
                  input_copy_streams=args.input_copy_streams if copy_streams is None else copy_streams,
                  callback_streams=callback_streams)
    tid = ctx.define("gauss_sobel", width=1024, height=1024, copy=copy or args.copy)
    ib, ob = ctx.in_bytes(tid), ctx.out_bytes(tid)
    stride = 128
    arr = make_jobs(ctx, tid, jobs_per_step, tin, pool, ib, tout, ob, stride)
    for _ in range(warmup):
        ctx.submit_many(tid, arr)
        ctx.drain()
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_s = []
    for _ in range(steps):
        ts = time.perf_counter()
        ctx.submit_many(tid, arr)
        ctx.drain()
        step_s.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.stats()
    times = ctx.job_times()
    return ctx, tid, dt, st, (times, step_s)


def verify(tout, n_jobs, pool_imgs, refs):
    """Every job's result vs the oracle of its pool image (outside any timed region)."""
    import oracle
    from paper_2606_05495_amd import _abi as A
    out = tout.numpy().reshape(-1, 128)[:n_jobs]
    hdr = out[:, :64].copy().view(A.OUT_HEADER_DTYPE).ravel()
    ok = bool(np.all(hdr["magic"] == A.SET_OUT_MAGIC) and np.all(hdr["canary_ok"] == 1))
    cnt = out[:, 64:68].copy().view(np.uint32).ravel()
    s = out[:, 68:72].copy().view(np.float32).ravel()
    bad = 0
    for j in range(n_jobs):
        r = refs[j % len(refs)]
        if abs(int(cnt[j]) - r["count"]) > r["band"] or abs(float(s[j]) - r["sum"]) > 1e-5 * abs(r["sum"]):
            bad += 1
    return ok and bad == 0, bad


def cpu_baseline(pool_imgs, passes):
    """The oracle as it stands, timed on this host's cores: a thread pool of
    C calls (ctypes releases the interpreter lock) over `passes` x the pool."""
    import oracle
    oracle.lib()
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    work = [pool_imgs[k % len(pool_imgs)] for k in range(passes * len(pool_imgs))]
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=ncores) as ex:
        list(ex.map(lambda im: oracle.gauss_sobel(im, want_images=False), work))
    dt = time.perf_counter() - t0
    single = pool_imgs[:min(16, len(pool_imgs))]
    t1 = time.perf_counter()
    for im in single:
        oracle.gauss_sobel(im, want_images=False)
    dt1 = time.perf_counter() - t1
    return {"value": round(len(work) / dt, 2), "unit": "jobs/s", "cores": ncores, "kind": "oracle",
            "sample": "%d jobs = %d passes over the 61 pool images (1024x1024 Gaussian->Sobel->threshold->count/sum, "
                      "float64 C oracle), thread pool of %d" % (len(work), passes, ncores),
            "single_thread_jobs_per_s": round(len(single) / dt1, 2), "cpu_model": cpu_model()}


def oracle_pool_rate(fn, items, label):
    """The oracle over `items` on every host core (thread pool of C calls that
    release the interpreter lock), and on one thread over a fifth of them."""
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=ncores) as ex:
        list(ex.map(fn, items))
    dt = time.perf_counter() - t0
    few = items[:max(1, len(items) // 5)]
    t1 = time.perf_counter()
    for it in few:
        fn(it)
    dt1 = time.perf_counter() - t1
    return {"value": round(len(items) / dt, 2), "unit": "jobs/s", "cores": ncores, "kind": "oracle", "sample": label,
            "single_thread_jobs_per_s": round(len(few) / dt1, 2)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def nearest_rank(values, p):
    """The p-th percentile by nearest rank: the smallest value with at least
    p% of the sample at or below it."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return None
    k = max(1, int(np.ceil(p / 100.0 * v.size)))
    return float(v[k - 1])


def link_probe(torch, chunk=64 << 20, total=1 << 30):
    """Host-to-device bandwidth of the link with nothing else running: the
    best of 2 and 4 streams, each issuing hipMemcpyAsync copies of 64 MiB
    from pinned memory (the DMA engines, as the jobs' input copies), 1 GiB in
    all per setting (less data leaves the ramp in the figure)."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    hip.hipMemcpyAsync.restype = ctypes.c_int
    h2d = 1  # hipMemcpyHostToDevice
    src = torch.empty(chunk * 4, dtype=torch.uint8, pin_memory=True)
    dst = torch.empty(chunk * 4, dtype=torch.uint8, device="cuda")
    best = 0.0
    for streams in (2, 4):
        sts = [torch.cuda.Stream() for _ in range(streams)]
        rounds = max(1, total // (chunk * streams))

        def burst(n):
            for _ in range(n):
                for i, st in enumerate(sts):
                    rc = hip.hipMemcpyAsync(dst.data_ptr() + i * chunk, src.data_ptr() + i * chunk, chunk, h2d,
                                            st.cuda_stream)
                    if rc != 0:
                        raise RuntimeError("hipMemcpyAsync failed: %d" % rc)
        burst(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        burst(rounds)
        torch.cuda.synchronize()
        best = max(best, chunk * streams * rounds / (time.perf_counter() - t0) / 1e9)
    return round(best, 2)


def traffic_for(kernel_name, workload="gauss_sobel_1024"):
    """HBM bytes (fetched + written) per launch from committed rocprofv3 counter
    runs of the cold launch loop, if they were taken on the current kernel
    source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2606_05495_amd", "csrc", "kernels.hip"), "rb").read()
        if rec.get("kernels_sha256") != hashlib.sha256(src).hexdigest():
            return None
        return rec["workloads"][workload]["kernels"][kernel_name]["total"]
    except Exception:
        return None


def copy_reference(ctx, torch, nbytes, reps, span=1 << 30):
    """A plain device copy moving the same bytes (half read, half written),
    rotating over about `span` bytes of sources and destinations so that, like
    the cold stage timing, every copy reads and writes HBM: the bandwidth HBM
    delivers at this transfer size.  The reference is the library's copy
    kernel (one 16-byte word per thread, every word in flight at once); the
    runtime's device-to-device copy (hipMemcpy's blit kernel, a small grid
    looping over the bytes) is slower at these sizes and given beside it."""
    from paper_2606_05495_amd.stage_probe import cold_copy_us
    half = max(16, (nbytes // 2 + 15) // 16 * 16)
    us = ctx.time_device_copy(2 * half, reps)
    rt = cold_copy_us(torch, half, reps, span)
    return {"bytes": 2 * half, "avg_us": round(us, 3), "GBps": round(2 * half / us / 1e3, 1),
            "kernel": "plain copy kernel, one 16-byte word per thread", "buffers": "rotating over %d MiB" % (span >> 20),
            "runtime_copy": {"avg_us": round(rt, 3), "GBps": round(2 * half / rt / 1e3, 1)}}


def _vec_persistent(args, torch, A, autotune, Context, js, vj, xd, yd, J, total_bytes, check):
    out = {}
    # ---- bucketed persistent batches, dispatched by SET
    ctx = Context(mode="set", workers=args.workers, slots=4, callback=args.callback, dispatchers=args.dispatchers)

    def define(block):
        return ctx.define("saxpy_batch", max_n=int(js["n"].max()), x_pool=xd, y_pool=yd, batch_max=args.batch_max,
                          tiles_max=args.tiles_max, copy=args.copy, block=block)

    cache = args.tune_cache or autotune.DEFAULT_CACHE
    tuning = None if (args.no_tune or args.retune) else autotune.load(cache)
    block = 0 if (args.no_tune or args.retune) else autotune.load_block(cache)
    if tuning is None and not args.no_tune:
        log("autotuning block size and buckets")
        tuning, block = autotune.tune_blocks(ctx, define, vj, calib=512, cache=cache, log=log)
    tid = define(block)
    res = np.zeros(J, np.float32)
    ctx.run_vector_jobs(tid, vj, res, tuning)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, nb = ctx.run_vector_jobs(tid, vj, res, tuning)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["persistent"] = {"jobs_per_s": round(J / dt, 1), "batches": int(nb), "verified": check(res),
                         "effective_GBps": round(total_bytes / dt / 1e9, 1), "tuned": tuning is not None,
                         "block": block or 256}
    ctx.close()
    return out


def bench_vectors(args, torch):
    """100,000 uneven vector jobs (n log-uniform in [4096, 4194304)) over two
    2^27-element device pools: bucketed persistent batches dispatched by SET vs
    per-job graphs (SET), the batch-synchronised graph baseline and the
    synchronous baseline.  Prints one JSON line."""
    out = vectors_section(args, torch)
    if args.only:
        print(json.dumps({"mode": args.only, "workload": "vectors", "jobs_per_s": out["per_job_" + args.only]["jobs_per_s"],
                          "verified": out["per_job_" + args.only]["verified"]}), flush=True)
        return
    p = out["persistent"]["jobs_per_s"]
    line = {"metric": METRIC, "workload": "vector jobs: %d uneven (n log-uniform [4096, 4194304)) SAXPY->tanh->sum"
            % args.vjobs, "value": p, "unit": "jobs/s", "n_gpus": 1, "dtype": "f32", "data": "synthetic",
            "higher_is_better": True, "vs_baseline": None}
    line.update(vectors_summary(out))
    line["modes"] = out
    line["config"] = {"workers": args.workers, "batch_max": args.batch_max, "tiles_max": args.tiles_max,
                      "copy": args.copy, "callback": args.callback, "dispatchers": args.dispatchers,
                      "tuned": out["persistent"]["tuned"]}
    print(json.dumps(line), flush=True)


def box_section(args, torch, reps=20):
    """The 64-job box/histogram workload: 256x256 uint8 images (seeded by job
    id) -> 3x3 zero-padded box sum -> floor(/9) -> 256-bin histogram, as the
    plain method runs it (synchronous launches, stream = job mod 4) and through
    SET (4 workers x 4 slots, 4 dispatcher threads), beside the batch-synchronised
    graph baseline (batch 8 over 4 workers x 2 slots) and the queue model; `reps`
    timed passes of the 64 jobs each, every histogram of every pass bit-exact
    against the oracle."""
    from paper_2606_05495_amd import synth
    from paper_2606_05495_amd.runtime import Context, pinned
    import oracle
    J = 64
    imgs = [synth.box_image(0, j) for j in range(J)]
    refs = [oracle.box_hist(im)[2] for im in imgs]
    tin, nin = pinned(J * 65536)
    nin[:] = np.concatenate([im.ravel() for im in imgs])
    out = {}
    # SET as for the other short-job workloads: completion words, four
    # dispatcher threads (a job's graph launch costs ~14 us of host time)
    for mode, slots, cb, nd in (("sync", 1, "event_poll", 1), ("set", 4, "host_flag", 4), ("batch", 2, "event_poll", 1),
                                ("queue", 1, "event_poll", 1)):
        ctx = Context(mode=mode, workers=4, slots=slots, callback=cb, dispatchers=nd,
                      batch_size=8 if mode == "batch" else 0)
        tid = ctx.define("box_hist", width=256, height=256, copy="kernels")
        ob = ctx.out_bytes(tid)
        tout, nout = pinned(J * 1152)
        arr = ctx.job_array(J)
        j = np.arange(J, dtype=np.uint64)
        arr["host_in"] = tin.data_ptr() + j * np.uint64(65536)
        arr["in_bytes"] = 65536
        arr["host_out"] = tout.data_ptr() + j * np.uint64(1152)
        arr["out_bytes"] = ob
        ctx.submit_many(tid, arr)
        ctx.drain()
        ok, each = True, []
        for _ in range(reps):
            nout[:] = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.submit_many(tid, arr)
            ctx.drain()
            torch.cuda.synchronize()
            each.append(time.perf_counter() - t0)
            o = nout.reshape(J, 1152)
            ok &= all(np.array_equal(o[k, 64:64 + 1024].view(np.uint32), refs[k]) for k in range(J))
        ctx.close()
        dt = float(np.median(each))
        out[mode] = {"jobs_per_s": round(J / dt, 1), "passes": reps, "verified_bit_exact": bool(ok),
                     "jobs_per_s_min": round(J / max(each), 1), "jobs_per_s_max": round(J / min(each), 1)}
    out["set_speedup_vs_sync"] = round(out["set"]["jobs_per_s"] / out["sync"]["jobs_per_s"], 3)
    out["set_speedup_vs_batch_sync"] = round(out["set"]["jobs_per_s"] / out["batch"]["jobs_per_s"], 3)
    out["set_speedup_vs_queue"] = round(out["set"]["jobs_per_s"] / out["queue"]["jobs_per_s"], 3)
    if not args.no_cpu:
        out["cpu_oracle"] = oracle_pool_rate(oracle.box_hist, imgs, "all 64 jobs (C oracle)")
    out["verified"] = all(out[m]["verified_bit_exact"] for m in ("sync", "set", "batch", "queue"))
    return out


def vectors_summary(out):
    """Speedups of the persistent batches and of per-job SET over the per-job baselines."""
    p = out["persistent"]["jobs_per_s"]
    r = {"persistent_jobs_per_s": p}
    for m in ("set", "batch", "sync", "queue"):
        if "per_job_" + m in out:
            r["per_job_%s_jobs_per_s" % m] = out["per_job_" + m]["jobs_per_s"]
    if "per_job_batch" in out:
        r["speedup_vs_batch_sync"] = round(p / out["per_job_batch"]["jobs_per_s"], 3)
        if "per_job_set" in out:
            r["per_job_set_speedup_vs_batch_sync"] = round(out["per_job_set"]["jobs_per_s"] /
                                                           out["per_job_batch"]["jobs_per_s"], 3)
    if "per_job_queue" in out and "per_job_set" in out:
        r["per_job_set_speedup_vs_queue"] = round(out["per_job_set"]["jobs_per_s"] / out["per_job_queue"]["jobs_per_s"], 3)
    if "per_job_sync" in out:
        r["speedup_vs_sync"] = round(p / out["per_job_sync"]["jobs_per_s"], 3)
    if "per_job_set" in out:
        r["speedup_vs_per_job_set"] = round(p / out["per_job_set"]["jobs_per_s"], 3)
    r["verified"] = all(v.get("verified", True) for v in out.values() if isinstance(v, dict))
    if "cpu_oracle" in out:
        r["cpu_oracle_jobs_per_s"] = out["cpu_oracle"]["value"]
        r["persistent_over_cpu_oracle"] = round(p / out["cpu_oracle"]["value"], 1)
    return r


_VEC_POOLS = {}


def vector_pools(torch):
    """The two 2^27-element device pools of the vector jobs (host copies kept
    for the oracle), generated once per process."""
    from paper_2606_05495_amd import synth
    if "p" not in _VEC_POOLS:
        L = synth.VEC_POOL_LEN
        log("generating vector pools (2 x %d floats)" % L)
        x = synth.vec_pool(0, "x", L)
        y = synth.vec_pool(0, "y", L)
        _VEC_POOLS["p"] = (x, y, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    return _VEC_POOLS["p"]


def vectors_section(args, torch, modes=("set", "batch", "sync", "queue")):
    """Runs the uneven vector workload; returns {persistent, per_job_<mode>}."""
    from paper_2606_05495_amd import _abi as A
    from paper_2606_05495_amd import autotune, synth
    from paper_2606_05495_amd.runtime import Context, pinned
    import oracle
    L = synth.VEC_POOL_LEN
    x, y, xd, yd = vector_pools(torch)
    J = args.vjobs
    js = synth.vec_jobs(0, J, pool_len=L)
    vj = np.zeros(J, dtype=A.VEC_JOB_DTYPE)
    for f in ("n", "a", "x_off", "y_off"):
        vj[f] = js[f]
    total_bytes = 8.0 * float(js["n"].sum())
    sample = np.arange(0, J, max(1, J // args.vsample))
    refs = {int(i): oracle.saxpy_tanh_sum(x[js["x_off"][i]:js["x_off"][i] + js["n"][i]],
                                          y[js["y_off"][i]:js["y_off"][i] + js["n"][i]], js["a"][i]) for i in sample}

    def check(res):
        return all(abs(float(res[i]) - S) <= oracle.vec_tolerance(S, E) for i, (S, E) in refs.items())

    out = {}
    if args.only:
        # traced runs: one per-job mode only
        modes = (args.only,)
    else:
        out.update(_vec_persistent(args, torch, A, autotune, Context, js, vj, xd, yd, J, total_bytes, check))
    for mode in modes:
        c = Context(mode=mode, workers=args.workers, slots=16 if mode == "set" else 1,
                    batch_size=args.batch if mode == "batch" else 0, callback=args.callback, dispatchers=args.dispatchers,
                    inflight=args.inflight)
        t2 = c.define("saxpy_tanh_sum", max_n=int(js["n"].max()), x_pool=xd, y_pool=yd, copy=args.copy)
        tout, nout = pinned(128 * J)
        arr = c.job_array(J)
        arr["host_out"] = tout.data_ptr() + np.arange(J, dtype=np.uint64) * 128
        arr["out_bytes"] = 68
        arr["n"] = js["n"]
        arr["a"] = js["a"]
        arr["x_off"] = js["x_off"]
        arr["y_off"] = js["y_off"]
        c.submit_many(t2, arr[:min(J, 2000)])
        c.drain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.submit_many(t2, arr)
        c.drain()
        torch.cuda.synchronize()
        dt2 = time.perf_counter() - t0
        r2 = nout.reshape(J, 128)[:, 64:68].copy().view(np.float32).ravel()
        out["per_job_" + mode] = {"jobs_per_s": round(J / dt2, 1), "verified": check(r2)}
        log("vectors per-job %s: %.0f jobs/s" % (mode, J / dt2))
        c.close()
    if not args.only and not args.no_cpu:
        K = min(J, 1000)
        items = [(x[js["x_off"][i]:js["x_off"][i] + js["n"][i]], y[js["y_off"][i]:js["y_off"][i] + js["n"][i]],
                  float(js["a"][i])) for i in range(K)]
        out["cpu_oracle"] = oracle_pool_rate(lambda t: oracle.saxpy_tanh_sum(*t), items,
                                             "the first %d jobs of the workload (float64 C oracle)" % K)
    return out


def bench_scan(args, torch):
    """Copy-engine-bound jobs: 8 MiB int32 H2D -> inclusive int64 scan -> 16 MiB
    D2H (pool of 31 inputs), SET at several stream counts with stealing on and
    off, against the batch-synchronised graph and synchronous baselines."""
    configs = [("set", w, st, args.copy) for w in (4, 8, 16) for st in (True, False)]
    configs += [(m, 8, False, cp) for m in ("batch", "sync", "queue") for cp in ("kernels", "async_in")]
    if args.only:
        # traced runs: one mode, 8 workers, the given copy mechanism
        configs = [(args.only, 8, args.only == "set", args.copy)]
    runs = scan_section(args, torch, configs)
    if args.only:
        r = runs[0]
        print(json.dumps({"mode": args.only, "workload": "scan", "jobs_per_s": r["jobs_per_s"], "verified": r["verified"],
                          "copy": r["copy"]}), flush=True)
        return
    line = {"metric": METRIC, "workload": "scan jobs: %d x (8 MiB int32 H2D -> int64 inclusive scan -> 16 MiB D2H)"
            % args.scan_jobs, "unit": "jobs/s", "n_gpus": 1, "dtype": "int64", "data": "synthetic",
            "higher_is_better": True, "vs_baseline": None}
    line.update(scan_summary(runs))
    line["value"] = line["best"]["jobs_per_s"]
    line["runs"] = runs
    line["config"] = {"copy": args.copy, "callback": args.callback, "dispatchers": args.dispatchers,
                      "inflight_per_worker": args.inflight, "input_copy_streams": args.input_copy_streams}
    print(json.dumps(line), flush=True)


def scan_summary(runs):
    """Best SET run (and SET at 8 workers with and without stealing) against each baseline's fastest run."""
    best = max((r for r in runs if r["mode"] == "set"), key=lambda r: r["jobs_per_s"])
    base = {m: max((r for r in runs if r["mode"] == m), key=lambda r: r["jobs_per_s"])
            for m in ("batch", "sync", "queue") if any(r["mode"] == m for r in runs)}
    out = {"best": best, "baselines_best": {m: {"jobs_per_s": r["jobs_per_s"], "copy": r["copy"]} for m, r in base.items()}}
    for m, r in base.items():
        out["speedup_vs_" + ("batch_sync" if m == "batch" else m)] = round(best["jobs_per_s"] / r["jobs_per_s"], 3)
    for steal in (True, False):
        s8 = [r for r in runs if r["mode"] == "set" and r["workers"] == 8 and r["stealing"] == steal]
        if s8 and "batch" in base:
            out["set8_%s_speedup_vs_batch_sync" % ("stealing" if steal else "no_stealing")] = round(
                s8[0]["jobs_per_s"] / base["batch"]["jobs_per_s"], 3)
    out["verified"] = all(r["verified"] for r in runs)
    return out


def scan_section(args, torch, configs, cpu_out=None):
    """Runs (mode, workers, stealing, copy) configurations of the scan workload; returns one record each.
    With cpu_out (a dict), the oracle's rate over the pool's inputs is stored there."""
    from paper_2606_05495_amd import synth
    from paper_2606_05495_amd.runtime import Context, pinned
    import oracle
    n = 1 << 21
    P = synth.SCAN_POOL
    log("generating scan pool (%d x %d int32)" % (P, n))
    pool = synth.scan_pool(0, P, n)
    tin, nin = pinned(P * 4 * n)
    nin.view(np.int32)[:] = pool.ravel()
    R = args.scan_ring
    ob = 64 + 8 * n
    ostride = (ob + 4095) // 4096 * 4096
    tout, nout = pinned(R * ostride)
    J = args.scan_jobs

    def job_array(ctx, tid, count):
        arr = ctx.job_array(count)
        j = np.arange(count, dtype=np.uint64)
        arr["host_in"] = tin.data_ptr() + (j % np.uint64(P)) * np.uint64(4 * n)
        arr["in_bytes"] = 4 * n
        arr["host_out"] = tout.data_ptr() + (j % np.uint64(R)) * np.uint64(ostride)
        arr["out_bytes"] = ob
        arr["n"] = n
        return arr

    def verify(count):
        for j in range(min(count, R)):
            o = nout[j * ostride + 64:j * ostride + ob].view(np.int64)
            if not np.array_equal(o, oracle.scan(pool[j % P])):
                return False
        return True

    runs = []
    for mode, workers, steal, copy in configs:
        ctx = Context(mode=mode, workers=workers, slots=4 if mode == "set" else 1, stealing=steal,
                      batch_size=min(args.batch, workers) if mode == "batch" else 0, callback=args.callback,
                      dispatchers=args.dispatchers, input_copy_streams=args.input_copy_streams,
                      inflight=args.inflight)
        tid = ctx.define("scan", max_n=n, copy=copy)
        warm = job_array(ctx, tid, min(R, J))
        ctx.submit_many(tid, warm)
        ctx.drain()
        ok = verify(min(R, J))
        arr = job_array(ctx, tid, J)
        ctx.reset_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.submit_many(tid, arr)
        ctx.drain()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.stats()
        runs.append({"mode": mode, "workers": workers, "stealing": steal, "copy": copy, "jobs_per_s": round(J / dt, 1),
                     "h2d_GBps": round(J * 4 * n / dt / 1e9, 2), "d2h_GBps": round(J * 8 * n / dt / 1e9, 2),
                     "stolen": int(st.stolen), "verified": ok})
        log(json.dumps(runs[-1]))
        ctx.close()
    if cpu_out is not None and not args.no_cpu:
        cpu_out.update(oracle_pool_rate(oracle.scan, [pool[k] for k in range(P)],
                                        "the %d pool inputs (2^21 int32 each, C oracle)" % P))
    return runs


def bench_sweep(args, torch):
    """Worker-count sweep (the batch size b of Sections 5.2 and 5.3): per-job
    vector jobs (the uneven vector workload's length distribution,
    device-resident inputs, two kernels and a 68-byte D2H each) through SET (b
    workers, 16 slots each up to b = 64 and 4 above, min(4, b) dispatcher
    threads), batch-sync (one graph of b chains per batch) and the queue model
    (b workers), at b = 1 .. 256; batch-sync also runs larger batches (64
    workers, ceil(b / 64) slots each).  Every point carries its untraced
    scheduling-overhead fraction (Eq. 1-4 with per-job times measured apart,
    see overhead_fraction).  Prints one JSON line."""
    from paper_2606_05495_amd import synth
    from paper_2606_05495_amd.runtime import Context, pinned
    import oracle
    L = synth.VEC_POOL_LEN
    x = synth.vec_pool(0, "x", L)
    y = synth.vec_pool(0, "y", L)
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y).cuda()
    J = args.sweep_jobs
    js = synth.vec_jobs(0, J, pool_len=L)
    refs = {int(i): oracle.saxpy_tanh_sum(x[js["x_off"][i]:js["x_off"][i] + js["n"][i]],
                                          y[js["y_off"][i]:js["y_off"][i] + js["n"][i]], js["a"][i])
            for i in range(0, J, max(1, J // 20))}
    tout, nout = pinned(128 * J)
    rows = []
    modes = ("set", "batch", "queue")
    if args.only:
        if args.only not in modes:
            raise SystemExit("--only for the sweep takes set, batch or queue")
        modes = (args.only,)
    model = None if args.only else job_time_model(args, torch, xd, yd, L)
    for b in [int(v) for v in args.sweep_b.split(",")]:
        for mode in modes:
            # SET and the queue model run b workers (at most 256); a batch graph
            # of b > 64 chains spans slots: 64 workers x ceil(b / 64) slots
            if mode != "batch" and b > 256:
                continue
            nw = min(b, 256) if mode != "batch" else min(b, 64)
            slots = 16 if mode == "set" else (-(-b // 64) if mode == "batch" else 1)
            if mode == "set" and b > 64:
                slots = 4  # 4 slots x b workers: the same in-flight depth per worker, fewer graph execs
            c = Context(mode=mode, workers=nw, slots=slots,
                        batch_size=b if mode == "batch" else 0, callback=args.callback,
                        dispatchers=min(args.dispatchers, nw), inflight=args.inflight)
            tid = c.define("saxpy_tanh_sum", max_n=int(js["n"].max()), x_pool=xd, y_pool=yd, copy=args.copy)
            arr = c.job_array(J)
            arr["host_out"] = tout.data_ptr() + np.arange(J, dtype=np.uint64) * 128
            arr["out_bytes"] = 68
            for f in ("n", "a", "x_off", "y_off"):
                arr[f] = js[f]
            c.submit_many(tid, arr[:min(J, 1000)])
            c.drain()
            each, ok = [], True
            for _ in range(args.sweep_repeats):
                nout[:] = 0
                c.reset_stats()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                c.submit_many(tid, arr)
                c.drain()
                torch.cuda.synchronize()
                each.append(time.perf_counter() - t0)
                res = nout.reshape(J, 128)[:, 64:68].copy().view(np.float32).ravel()
                ok &= all(abs(float(res[i]) - S) <= oracle.vec_tolerance(S, E) for i, (S, E) in refs.items())
            st = c.stats()
            c.close()
            dt = float(np.median(each))
            row = {"b": b, "mode": mode, "jobs_per_s": round(J / dt, 1), "verified": bool(ok),
                   "jobs_per_s_each": [round(J / t, 1) for t in each],
                   "host_sync_ms": round(st.host_ns_sync / 1e6, 2), "stolen": int(st.stolen), "T_measured_ms": round(dt * 1e3, 3)}
            if model is not None:
                row.update(overhead_fraction(model, js["n"], b, dt))
            rows.append(row)
            log("b=%d %s %.0f jobs/s%s" % (b, mode, J / dt, "" if model is None else
                                          ", overhead fraction %.3f (Eq. 1 per batch), %.3f (serial)" %
                                          (row["overhead_fraction_eq1"], row["overhead_fraction_serial"])))
    table = {}
    frac = {}
    for r in rows:
        table.setdefault(r["b"], {})[r["mode"]] = r["jobs_per_s"]
        if "overhead_fraction_eq1" in r:
            frac.setdefault(r["b"], {})[r["mode"]] = {"eq1": r["overhead_fraction_eq1"],
                                                      "serial": r["overhead_fraction_serial"]}
    line = {"metric": METRIC, "workload": "worker-count sweep, %d per-job vector jobs per point" % J,
            "unit": "jobs/s", "n_gpus": 1, "dtype": "f32", "data": "synthetic", "higher_is_better": True,
            "vs_baseline": None, "table": table, "overhead_fraction": frac, "job_time_model": model,
            "set_over_batch": {b: round(t["set"] / t["batch"], 3) for b, t in table.items() if "set" in t and "batch" in t},
            "set_over_queue": {b: round(t["set"] / t["queue"], 3) for b, t in table.items() if "set" in t and "queue" in t},
            "runs": rows, "config": {"callback": args.callback, "dispatchers": args.dispatchers, "copy": args.copy}}
    print(json.dumps(line), flush=True)


def job_time_model(args, torch, xd, yd, L, reps=64):
    """Untraced per-job times of the per-job vector pipeline for Eq. 1: t_k(n)
    (the stage kernels back to back) at n = 2^12 .. 2^22, and t_in / t_out (the
    job's copies), each the mean over `reps` launches rotating over 64 slots
    that hold jobs of that length at different pool windows (so large jobs
    read from HBM, as in the run)."""
    from paper_2606_05495_amd import _abi as A
    from paper_2606_05495_amd.runtime import Context, pinned
    W = 64
    c = Context(mode="sync", workers=W, slots=1)
    tid = c.define("saxpy_tanh_sum", max_n=1 << 22, x_pool=xd, y_pool=yd, copy=args.copy)
    nst = len(c.stage_info(tid))
    tout, _ = pinned(128 * W)
    rng = np.random.default_rng(3)
    tk = {}
    for e in range(12, 23):
        n = 1 << e
        for w in range(W):
            c.submit(tid, host_out=tout.data_ptr() + 128 * w, out_bytes=68, n=n, a=1.0,
                     x_off=int(64 * rng.integers(0, (L - n) // 64)), y_off=int(64 * rng.integers(0, (L - n) // 64)))
        c.drain()
        tk[n] = sum(c.time_stage(tid, s_, -1, reps) for s_ in range(nst))
    t_in = c.time_stage(tid, A.SET_STAGE_INPUT_COPY, -1, reps)
    t_out = c.time_stage(tid, A.SET_STAGE_OUTPUT_COPY, -1, reps)
    c.close()
    return {"t_k_us": {str(n): round(v, 3) for n, v in tk.items()}, "t_in_us": round(t_in, 3),
            "t_out_us": round(t_out, 3), "copy": args.copy, "reps": reps, "slots": W}


def model_tk(model, n):
    """t_k(n) by linear interpolation in n between the measured powers of two."""
    pts = sorted((int(k), v) for k, v in model["t_k_us"].items())
    ns = np.array([p[0] for p in pts], np.float64)
    ts = np.array([p[1] for p in pts], np.float64)
    return np.interp(np.asarray(n, np.float64), ns, ts)


def overhead_fraction(model, n, b, T_measured_s):
    """Scheduling-overhead fraction t_schedule / T_measured (Section 5.3, Eq. 4)
    with T_ideal from Eq. 1 per batch of b consecutive jobs in submission order:
    the batch's input copies back to back plus the largest kernel + output
    copy time in it (for identical jobs exactly b t_in + t_k + t_out).  The b = 1
    reading (every job's copies and kernels back to back, no overlap) beside it."""
    tk = model_tk(model, n)
    t_in, t_out = model["t_in_us"], model["t_out_us"]
    J = len(tk)
    ideal = 0.0
    for i in range(0, J, b):
        seg = tk[i:i + b]
        ideal += len(seg) * t_in + float(seg.max()) + t_out
    serial = float(J * (t_in + t_out) + tk.sum())
    T = T_measured_s * 1e6
    return {"T_ideal_eq1_ms": round(ideal / 1e3, 3), "overhead_fraction_eq1": round(1.0 - ideal / T, 4),
            "T_ideal_serial_ms": round(serial / 1e3, 3), "overhead_fraction_serial": round(1.0 - serial / T, 4)}


def bench_hotspot(args, torch):
    """Thermal-grid jobs (a memory-bound iterative workload): H2D of a
    temperature and a power grid -> K explicit heat steps, one kernel each ->
    D2H of the final grid.  SET against batch-sync, synchronous and the queue
    model on the same jobs.  Prints one JSON line."""
    from paper_2606_05495_amd import synth
    from paper_2606_05495_amd.runtime import Context, pinned
    import oracle
    h = w = args.hot_side
    K, J, P = args.hot_steps, args.hot_jobs, 16
    grids = [synth.hotspot_input(0, k, h, w) for k in range(P)]
    refs = [oracle.hotspot(t0, p, K) for t0, p in grids]
    ib, ob = 8 * h * w, 64 + 4 * h * w
    istride, ostride = (ib + 255) // 256 * 256, (ob + 255) // 256 * 256
    tin, nin = pinned(istride * P)
    for i, (t0, p) in enumerate(grids):
        nin[i * istride:i * istride + ib].view(np.float32)[:] = np.concatenate([t0.ravel(), p.ravel()])
    R = 256  # output ring
    tout, nout = pinned(ostride * R)
    out = {}
    # SET with the configured copy mechanism; each baseline with every one
    # (scored by its fastest)
    runs = [("set", args.copy)] if not args.only else [(args.only, args.copy)]
    if not args.only:
        runs += [(m, cp) for m in ("batch", "sync", "queue") for cp in ("kernels", "async_in")]
    for mode, copy in runs:
        c = Context(mode=mode, workers=args.workers, slots=args.slots if mode == "set" else 1,
                    batch_size=args.batch if mode == "batch" else 0, callback=args.callback,
                    dispatchers=args.dispatchers, inflight=args.inflight,
                    input_copy_streams=args.input_copy_streams)
        tid = c.define("hotspot", width=w, height=h, max_n=K, copy=copy)
        j = np.arange(J, dtype=np.uint64)
        arr = c.job_array(J)
        arr["host_in"] = tin.data_ptr() + (j % np.uint64(P)) * np.uint64(istride)
        arr["in_bytes"] = ib
        arr["host_out"] = tout.data_ptr() + (j % np.uint64(R)) * np.uint64(ostride)
        arr["out_bytes"] = ob
        c.submit_many(tid, arr[:min(J, 2 * R)])
        c.drain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.submit_many(tid, arr)
        c.drain()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        c.close()
        # the ring holds the last R jobs: job J - R + i sits in ring entry (J - R + i) % R
        ok = True
        for i in range(min(R, J)):
            jj = J - min(R, J) + i
            o = nout[(jj % R) * ostride + 64:(jj % R) * ostride + ob].view(np.float32).reshape(h, w)
            ref = refs[jj % P]
            ok &= bool(np.max(np.abs(o - ref)) <= oracle.hotspot_tolerance(ref, K))
        r = {"jobs_per_s": round(J / dt, 1), "verified": ok, "copy": copy}
        log("hotspot %s %s %.0f jobs/s" % (mode, copy, J / dt))
        if mode not in out or r["jobs_per_s"] > out[mode]["jobs_per_s"]:
            out[mode] = dict(r, verified=ok and out.get(mode, {}).get("verified", True))
        else:
            out[mode]["verified"] = out[mode]["verified"] and ok
        out.setdefault("by_copy", {})["%s_%s" % (mode, copy)] = r["jobs_per_s"]
    if args.only:
        print(json.dumps({"mode": args.only, "workload": "hotspot", **out[args.only]}), flush=True)
        return
    v = out["set"]["jobs_per_s"]
    line = {"metric": METRIC, "workload": "thermal grid: %d jobs, %dx%d float32, %d steps per job" % (J, h, w, K),
            "value": v, "unit": "jobs/s", "n_gpus": 1, "dtype": "f32", "data": "synthetic",
            "higher_is_better": True, "vs_baseline": None,
            "speedup_vs_batch_sync": round(v / out["batch"]["jobs_per_s"], 3),
            "speedup_vs_sync": round(v / out["sync"]["jobs_per_s"], 3),
            "speedup_vs_queue": round(v / out["queue"]["jobs_per_s"], 3),
            "modes": out, "config": {"workers": args.workers, "slots": args.slots, "batch": args.batch,
                                     "callback": args.callback, "dispatchers": args.dispatchers, "copy": args.copy,
                                     "inflight_per_worker": args.inflight}}
    print(json.dumps(line), flush=True)


def bench_serve(args, torch):
    """Open-loop serving: Poisson arrivals at each rate for a fixed window; half
    image jobs (Gaussian/Sobel at 256^2, 512^2, 1024^2, 2048^2, uniform) and
    half vector jobs (as the uneven vector family), under an 8 GB
    device-memory admission cap.  Latency = arrival -> result in host memory."""
    results = serve_section(args, torch)
    line = {"metric": METRIC, "workload": "serving: Poisson arrivals, 50%% images {256,512,1024,2048}^2 + 50%% "
            "vector jobs, %.0f GB admission cap, %.0f s window" % (args.mem_budget / 1e9, args.serve_seconds),
            "value": results[0]["throughput_jobs_per_s"], "unit": "jobs/s", "n_gpus": 1, "dtype": "f32",
            "data": "synthetic", "higher_is_better": True, "vs_baseline": None, "rates": results,
            "config": {"workers": args.workers, "slots": args.slots, "copy": args.copy, "callback": args.callback,
                       "dispatchers": args.dispatchers, "inflight_per_worker": args.inflight,
                       "image_pool_per_size": args.serve_pool}}
    print(json.dumps(line), flush=True)


def serve_section(args, torch):
    """Runs the serving workload at each of args.rates; returns one record per rate."""
    from paper_2606_05495_amd import _abi as A
    from paper_2606_05495_amd import autotune, synth
    from paper_2606_05495_amd.runtime import Context, pinned
    import oracle
    sides = synth.SERVE_SIDES
    P = args.serve_pool
    log("generating serving pools (%d images per size)" % P)
    imgs = {s_: synth.serve_image_pool(0, s_, count=P) for s_ in sides}
    off, offs = 0, {}
    for s_ in sides:
        offs[s_] = off
        off += P * 4 * s_ * s_
    tin, nin = pinned(off)
    for s_ in sides:
        nin[offs[s_]:offs[s_] + P * 4 * s_ * s_].view(np.float32)[:] = imgs[s_].ravel()
    L = synth.VEC_POOL_LEN
    xh, yh, xd, yd = vector_pools(torch)
    img_refs = {}

    def check_sample(req, isimg, side, mix, done, vres, nout, rate, count=200):
        """A seeded sample of completed requests of each kind against the oracle."""
        rng = np.random.default_rng(int(rate))
        ok = True
        idx_img = np.flatnonzero(isimg & (done > 0))
        idx_vec = np.flatnonzero(~isimg & (done > 0))
        picks_img = rng.choice(idx_img, min(count, idx_img.size), replace=False) if idx_img.size else []
        picks_vec = rng.choice(idx_vec, min(count, idx_vec.size), replace=False) if idx_vec.size else []
        for i in picks_img:
            key = (int(side[i]), int(mix["pool_idx"][i] % P))
            if key not in img_refs:
                img_refs[key] = oracle.gauss_sobel(imgs[key[0]][key[1]], want_images=False)
            r = img_refs[key]
            o = nout[i * 128:(i + 1) * 128]
            ok &= abs(int(o[64:68].view(np.uint32)[0]) - r["count"]) <= r["band"]
            ok &= abs(float(o[68:72].view(np.float32)[0]) - r["sum"]) <= 1e-5 * abs(r["sum"])
        for i in picks_vec:
            n_, xo, yo = int(req["n"][i]), int(req["x_off"][i]), int(req["y_off"][i])
            S, E = oracle.saxpy_tanh_sum(xh[xo:xo + n_], yh[yo:yo + n_], req["a"][i])
            ok &= abs(float(vres[i]) - S) <= oracle.vec_tolerance(S, E)
        return bool(ok), len(picks_img) + len(picks_vec)

    results = []
    for rate in [float(r) for r in args.rates.split(",")]:
        ctx = Context(mode="set", workers=args.workers, slots=args.slots, mem_budget=int(args.mem_budget),
                      callback=args.callback, inflight=args.inflight, dispatchers=args.dispatchers,
                      input_copy_streams=args.input_copy_streams)
        timg = {s_: ctx.define("gauss_sobel", width=s_, height=s_, copy=args.copy) for s_ in sides}
        tvec = ctx.define("saxpy_batch", max_n=4194303, x_pool=xd, y_pool=yd, batch_max=args.batch_max,
                          tiles_max=args.tiles_max, copy=args.copy,
                          block=0 if args.no_tune else autotune.load_block(args.tune_cache or autotune.DEFAULT_CACHE))
        tuning = None if args.no_tune else autotune.load(args.tune_cache or autotune.DEFAULT_CACHE)
        arr = synth.poisson_arrivals(int(rate), rate, args.serve_seconds)
        n = len(arr)
        mix = synth.serve_mix(int(rate), n)
        vj = synth.vec_jobs(int(rate), n, pool_len=L, cfg=synth.CFG_SERVE)
        req = np.zeros(n, dtype=A.REQUEST_DTYPE)
        req["t_arrival_ns"] = (arr * 1e9).astype(np.uint64)
        req["worker_hint"] = -1
        isimg = mix["kind"] == 0
        side = np.array(sides)[mix["side_idx"]]
        tout, nout = pinned(128 * n)
        req["template_id"] = np.where(isimg, [timg[s_] for s_ in side], tvec)
        base = np.array([offs[s_] for s_ in side], dtype=np.uint64)
        req["host_in"] = np.where(isimg, tin.data_ptr() + base + (mix["pool_idx"] % P).astype(np.uint64) *
                                  (4 * side * side).astype(np.uint64), 0)
        req["in_bytes"] = np.where(isimg, 4 * side * side, 0)
        req["host_out"] = np.where(isimg, tout.data_ptr() + np.arange(n, dtype=np.uint64) * 128, 0)
        req["out_bytes"] = np.where(isimg, 72, 0)
        for f in ("n", "a", "x_off", "y_off"):
            req[f] = np.where(isimg, 0, vj[f])
        vres = np.zeros(n, np.float32)
        cfg = A.set_serve_config()
        if tuning is not None:
            cfg.tuning = ctypes.pointer(tuning)
        log("serving %.0f jobs/s: %d requests over %.1f s" % (rate, n, args.serve_seconds))
        done, st = A.set_serve(ctx.h, req, cfg, vres)
        ok = done > 0
        lat = (done[ok].astype(np.float64) - req["t_arrival_ns"][ok].astype(np.float64)) / 1e3
        span = (st.t_end_ns - st.t_start_ns) / 1e9
        h2d_offered = float(np.sum(req["in_bytes"])) / args.serve_seconds / 1e9
        res = {"rate": rate, "requests": int(n), "completed": int(st.completed), "failed": int(st.failed),
               "throughput_jobs_per_s": round(st.completed / span, 1) if span > 0 else None,
               "p50_us": round(nearest_rank(lat, 50), 1), "p99_us": round(nearest_rank(lat, 99), 1),
               "p50_image_us": round(nearest_rank(lat[isimg[ok]], 50), 1),
               "p99_image_us": round(nearest_rank(lat[isimg[ok]], 99), 1),
               "p50_vector_us": round(nearest_rank(lat[~isimg[ok]], 50), 1),
               "p99_vector_us": round(nearest_rank(lat[~isimg[ok]], 99), 1),
               "max_backlog": int(st.max_backlog), "vec_batches": int(st.vec_batches),
               "offered_h2d_GBps": round(h2d_offered, 1), "mem_high_water_GB": round(ctx.stats().mem_high_water / 1e9, 2),
               "drain_after_window_s": round(span - args.serve_seconds, 3)}
        res["verified"], res["checked"] = check_sample(req, isimg, side, mix, done, vres, nout, rate)
        log(json.dumps(res))
        results.append(res)
        ctx.close()
    return results


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--jobs", type=int, default=10000, help="jobs per step")
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--inflight", type=int, default=None,
                    help="SET launch permits per worker (default 1 with async_in copies, else the library's "
                         "min(2, d))")
    ap.add_argument("--spin-us", type=int, default=0)
    ap.add_argument("--dispatchers", type=int, default=None,
                    help="SET dispatcher threads (default: 1 for the image workload; for the thermal grid 2 up to "
                         "256^2 and 1 above; 4 otherwise)")
    ap.add_argument("--callback", default=None, choices=["event_chain", "same_stream", "event_poll", "host_flag", "event_blocking"],
                    help="SET completion mechanism (default event_poll with async_in copies, host_flag otherwise)")
    ap.add_argument("--copy", default=None, choices=["nodes", "kernels", "async_in"],
                    help="job copies: graph memcpy nodes, small-grid copy kernels, or the input by hipMemcpyAsync "
                         "ahead of the graph (default: async_in for the image, scan and thermal-grid workloads, "
                         "kernels otherwise); their baselines run every mechanism and keep their fastest")
    ap.add_argument("--input-copy-streams", type=int, default=None,
                    help="streams carrying the async input copies (default 0: each worker's own stream)")
    ap.add_argument("--baseline-steps", type=int, default=1)
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-passes", type=int, default=15)
    ap.add_argument("--stage-reps", type=int, default=200)
    ap.add_argument("--workload", choices=["images", "vectors", "serve", "scan", "sweep", "hotspot"], default="images")
    ap.add_argument("--hot-side", type=int, default=256)
    ap.add_argument("--hot-steps", type=int, default=16)
    ap.add_argument("--hot-jobs", type=int, default=10000)
    ap.add_argument("--sweep-b", default="1,2,4,8,16,32,64,128,256,512,1024,2048,4096",
                    help="batch sizes b of the sweep workload (SET and the queue model stop at 256)")
    ap.add_argument("--sweep-jobs", type=int, default=20000)
    ap.add_argument("--sweep-repeats", type=int, default=3, help="timed passes per sweep point (median reported)")
    ap.add_argument("--scan-jobs", type=int, default=20000)
    ap.add_argument("--scan-ring", type=int, default=48)
    ap.add_argument("--rates", default="2000,10000,40000")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-pool", type=int, default=16)
    ap.add_argument("--section-serve-seconds", type=float, default=3.0,
                    help="image workload: window of each rate in the serving section of the default line")
    ap.add_argument("--mem-budget", type=float, default=8e9)
    ap.add_argument("--vjobs", type=int, default=100000)
    ap.add_argument("--vsample", type=int, default=400)
    ap.add_argument("--batch-max", type=int, default=1024)
    ap.add_argument("--tiles-max", type=int, default=16384)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--retune", action="store_true", help="vector workloads: tune block, item sizes and grids afresh")
    ap.add_argument("--tune-cache", default=None, help="tuning cache file (default: the package's tuning/vec_batch.json)")
    ap.add_argument("--image-pool", type=int, default=61, help="distinct images the jobs cycle through")
    ap.add_argument("--mechanisms", default="event_poll,event_chain,event_chain_per_worker,event_blocking",
                    help="SET completion mechanisms the image workload also runs (comma list; empty: none)")
    ap.add_argument("--mech-steps", type=int, default=3)
    ap.add_argument("--no-sections", action="store_true",
                    help="image workload: skip the vector and scan sections of the default line")
    ap.add_argument("--no-trace", action="store_true", help="image workload: no traced child runs")
    ap.add_argument("--trace-modes", default="set,batch,queue")
    ap.add_argument("--trace-batch-copy", default="kernels", choices=["nodes", "kernels", "async_in"],
                    help="copy mechanism of the traced batch-sync child (its fastest in every measured run)")
    ap.add_argument("--trace-jobs", type=int, default=2000)
    ap.add_argument("--trace-timeout", type=int, default=240)
    ap.add_argument("--only", choices=["set", "batch", "sync", "queue"], default=None,
                    help="run one mode only (for traced runs); prints its line")
    args = ap.parse_args()
    raw = argparse.Namespace(**vars(args))
    apply_defaults(args)
    main_with(args, raw)


def apply_defaults(args):
    """Per-workload defaults of the options left unset (args.workload decides)."""
    if args.copy is None:
        args.copy = "async_in" if args.workload in ("images", "scan", "hotspot", "serve") else "kernels"
    # With DMA input copies the fastest measured SET settings are one job in
    # flight per worker (a second job's copy waits behind its stream's graph,
    # and that wait shares a hardware queue with other streams' kernels) and
    # completion by event polling (no completion-word kernel per job).  With
    # copy kernels, two in flight and completion words.
    if args.input_copy_streams is None:
        args.input_copy_streams = 0
    if args.inflight is None:
        args.inflight = 1 if args.copy == "async_in" else 0
    if args.callback is None:
        # Serving keeps completion words with DMA input copies: at 10k
        # requests/s its p99 is lower with them than with event polling.
        args.callback = "event_poll" if args.copy == "async_in" and args.workload != "serve" else "host_flag"
    if args.dispatchers is None:
        # As few dispatcher threads as the launch rate allows: with several,
        # launches onto streams that share a hardware queue interleave, and a
        # graph's wait on its DMA input copy can then sit between another
        # job's kernels (traced: 50-66 us gaps inside jobs with 4 threads,
        # none with 1).  One thread sustains about 30k launches/s of the
        # 18-node thermal-grid graph: enough for 1024^2 images (13.6k jobs/s)
        # and 512^2 grids (22k), not for 256^2 grids (39k), which take two.
        # Per-job vector dispatch is host-bound and keeps four.
        if args.workload == "images":
            args.dispatchers = 1
        elif args.workload == "hotspot":
            args.dispatchers = 1 if args.hot_side >= 512 else 2
        else:
            args.dispatchers = 4
    return args


def section_args(raw, workload, **overrides):
    """The options another workload's section runs with: the command line's
    explicit settings that apply to it, then that workload's defaults."""
    ns = argparse.Namespace(**vars(raw))
    ns.workload = workload
    ns.only = None
    for k in ("copy", "callback", "dispatchers", "inflight", "input_copy_streams"):
        setattr(ns, k, None)  # the image workload's explicit settings are not carried over
    for k, v in overrides.items():
        setattr(ns, k, v)
    return apply_defaults(ns)


TRACE_KEYS = ("mean_gap", "mean_kernel_gap", "mean_positive_kernel_gap", "gpu_idle_fraction", "compute_idle_fraction",
              "h2d_idle_fraction", "span", "kernels", "h2d_copies", "mean_inter_batch_us")


def traced_timelines(args, modes):
    """Kernel gap and GPU-idle fraction of each mode, from rocprofv3 kernel and
    copy traces of a child run of this script (`--only MODE`, a short run of
    the same image jobs).  Called before this process touches the GPU, so the
    children have the device to themselves.  Returns {mode: metrics} plus the
    command; a mode whose trace could not be taken carries an "error"."""
    import shutil
    import subprocess
    import tempfile
    from paper_2606_05495_amd import trace
    prof = shutil.which("rocprofv3") or ("/opt/rocm/bin/rocprofv3" if os.path.exists("/opt/rocm/bin/rocprofv3") else None)
    out = {"modes": {}, "jobs_per_step": args.trace_jobs, "steps": 2}
    if not prof:
        out["error"] = "rocprofv3 not found"
        return out
    env = dict(os.environ, TMPDIR="/tmp")
    for mode in modes:
        d = tempfile.mkdtemp(prefix="set_trace_%s_" % mode, dir="/tmp")
        # each mode traced with the copy mechanism it is scored with: SET's own,
        # the baselines' fastest (copy kernels for batch-sync, DMA for the queue model)
        copy = args.copy if mode == "set" else {"batch": args.trace_batch_copy, "queue": "async_in"}.get(mode, "kernels")
        child = [sys.executable, os.path.abspath(__file__), "--only", mode, "--steps", "2", "--warmup", "1",
                 "--jobs", str(args.trace_jobs), "--image-pool", "8", "--baseline-steps", "2", "--no-cpu",
                 "--callback", args.callback, "--copy", copy, "--dispatchers", str(args.dispatchers),
                 "--inflight", str(args.inflight), "--workers", str(args.workers), "--slots", str(args.slots),
                 "--batch", str(args.batch)]
        cmd = [prof, "--kernel-trace", "--memory-copy-trace", "--output-format", "csv", "-d", d, "-o", "trace", "--"] + child
        out["command"] = " ".join(["rocprofv3", "--kernel-trace", "--memory-copy-trace", "--output-format", "csv",
                                   "-d", "DIR", "-o", "trace", "--", "python3", "bench.py"] + child[2:])
        log("traced child: %s" % mode)
        try:
            r = subprocess.run(cmd, cwd="/tmp", env=env, timeout=args.trace_timeout, stdout=subprocess.PIPE,
                               stderr=subprocess.PIPE, text=True)
            line = [l for l in r.stdout.splitlines() if l.startswith("{")]
            # rocprofv3 may exit non-zero after a complete run; the child's own
            # line and complete CSVs decide
            if not line:
                out["modes"][mode] = {"error": "child printed no result (rc %d): %s" % (r.returncode, r.stderr[-400:])}
                continue
            res = json.loads(line[-1])
            m = trace.analyze_dir(d, batch=args.batch if mode == "batch" else 0, library_window=True)
            rec = {k: m.get(k) for k in TRACE_KEYS}
            rec["traced_jobs_per_s"] = res.get("jobs_per_s")
            rec["copy"] = copy
            rec["verified"] = res.get("verified")
            out["modes"][mode] = rec
        except subprocess.TimeoutExpired:
            out["modes"][mode] = {"error": "traced child timed out after %d s" % args.trace_timeout}
        except Exception as e:  # a malformed trace must not take the benchmark down
            out["modes"][mode] = {"error": "%s: %s" % (type(e).__name__, e)}
        finally:
            shutil.rmtree(d, ignore_errors=True)
    return out


def run_mechanisms(args, tin, tout, pool, torch, imgs, refs):
    """The same image jobs in SET with each other completion mechanism (Algorithm 3's
    release path), a short run each: jobs/s, and the host CPU time the process used
    per second of the run (a spinning completion thread shows as about one core).
    "event_chain" shares one callback stream among the workers;
    "event_chain_per_worker" gives each worker its own."""
    out = {}
    for name in [c for c in args.mechanisms.split(",") if c and c != args.callback]:
        per_worker = name == "event_chain_per_worker"
        cb = "event_chain" if per_worker else name
        log("SET with %s: %d jobs x %d steps" % (name, args.jobs, args.mech_steps))
        tout.zero_()
        c0 = time.process_time()
        w0 = time.perf_counter()
        ctx, _, dt, st, _ = run_mode("set", args, args.jobs, args.mech_steps, 1, tin, tout, pool, torch, callback=cb,
                                     callback_streams=args.workers if per_worker else 0)
        cpu = (time.process_time() - c0) / (time.perf_counter() - w0)
        ctx.close()
        ok, bad = verify(tout, args.jobs, imgs, refs)
        out[name] = {"jobs_per_s": round(args.jobs * args.mech_steps / dt, 1), "verified": ok, "wrong_jobs": int(bad),
                     "steps": args.mech_steps, "host_cpu_s_per_s": round(cpu, 2),
                     "host_us_per_job_launch": round(st.host_ns_launch / 1e3 / max(1, st.completed), 2)}
    return out


def main_with(args, raw):
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the job path shards by running one independent scheduler per GPU, "
              "and runs on more than one GPU are not part of this build (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    # Traced child runs first: this process has not touched the GPU yet.
    traced = None
    if args.workload == "images" and args.only is None and not args.no_trace:
        traced = traced_timelines(args, [m for m in args.trace_modes.split(",") if m])
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU (HIP device)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "vectors":
        bench_vectors(args, torch)
        return
    if args.workload == "serve":
        bench_serve(args, torch)
        return
    if args.workload == "scan":
        bench_scan(args, torch)
        return
    if args.workload == "sweep":
        bench_sweep(args, torch)
        return
    if args.workload == "hotspot":
        bench_hotspot(args, torch)
        return
    from paper_2606_05495_amd import synth
    from paper_2606_05495_amd.runtime import pinned
    import oracle

    pool = args.image_pool
    log("generating %d pool images" % pool)
    imgs = synth.image_pool(0, pool)
    ib = 4 * 1024 * 1024
    tin, nin = pinned(ib * pool)
    nin.view(np.float32)[:] = imgs.ravel()
    tout, _ = pinned(128 * args.jobs)
    refs = [oracle.gauss_sobel(imgs[k], want_images=False) for k in range(pool)]

    if args.only in ("batch", "sync", "queue"):
        log("%s only: %d jobs x %d steps" % (args.only, args.jobs, args.steps))
        c2, _, dt2, st2, _ = run_mode(args.only, args, args.jobs, args.steps, args.warmup, tin, tout, pool, torch)
        c2.close()
        ok2, _ = verify(tout, args.jobs, imgs, refs)
        print(json.dumps({"mode": args.only, "jobs_per_s": round(args.jobs * args.steps / dt2, 1),
                          "verified": ok2}), flush=True)
        return
    log("SET mode: %d jobs x %d steps" % (args.jobs, args.steps))
    c0, w0 = time.process_time(), time.perf_counter()
    ctx, tid, dt, st, (times, step_s) = run_mode("set", args, args.jobs, args.steps, args.warmup, tin, tout, pool, torch,
                                       callback=args.callback)
    set_cpu = (time.process_time() - c0) / (time.perf_counter() - w0)
    n_total = args.jobs * args.steps
    set_jps = n_total / dt
    set_ok, set_bad = verify(tout, args.jobs, imgs, refs)
    lat_dev = (times["t_done"] - times["t_launch"]) / 1e3
    lat_sub = (times["t_done"] - times["t_submit"]) / 1e3
    if args.only == "set":
        ctx.close()
        print(json.dumps({"mode": "set", "jobs_per_s": round(set_jps, 1), "verified": bool(set_ok)}), flush=True)
        return

    # Dominant kernel of the chain, timed with HIP events on the stream its
    # launches run on.  Cold: launch r works on slot r mod 128 of the
    # template (128 slots x 13 MiB, far beyond the 256 MB of last-level
    # cache), so every launch reads and writes HBM.  Warm: every launch on
    # one slot, whose 8 MiB stay cached (the figure the first measurements
    # reported, kept for comparison).
    stages = ctx.stage_info(tid)
    stage_us = [ctx.time_stage(tid, i, -1, args.stage_reps) for i in range(len(stages))]
    warm_us = [ctx.time_stage(tid, i, 0, args.stage_reps) for i in range(len(stages))]
    dom = int(np.argmax(stage_us))
    dom_name, dom_bytes = stages[dom]
    achieved = dom_bytes / (stage_us[dom] * 1e-6) / 1e9
    # Eq. 1's per-job terms, untraced: the job's input copy (DMA from pinned
    # memory), its stage kernels (cold, as above) and its output copy
    from paper_2606_05495_amd import _abi as A
    eq1 = {"t_in_us": round(ctx.time_stage(tid, A.SET_STAGE_INPUT_COPY, -1, 50), 3),
           "t_k_us": round(float(sum(stage_us)), 3),
           "t_out_us": round(ctx.time_stage(tid, A.SET_STAGE_OUTPUT_COPY, -1, 50), 3)}
    ref = copy_reference(ctx, torch, int(dom_bytes), args.stage_reps)
    ctx.close()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic_for(dom_name),
                "kernel": dom_name, "bytes_per_launch": int(dom_bytes), "avg_us": round(stage_us[dom], 3),
                "launches": args.stage_reps, "buffers": "cold: launch r on slot r mod %d" % (args.workers * args.slots),
                "stages_us": {n: round(u, 3) for (n, _), u in zip(stages, stage_us)},
                "warm_one_slot": {"avg_us": round(warm_us[dom], 3),
                                  "achieved": round(dom_bytes / (warm_us[dom] * 1e-6) / 1e9, 1),
                                  "stages_us": {n: round(u, 3) for (n, _), u in zip(stages, warm_us)}},
                "copy_same_bytes": ref, "frac_of_copy": round(achieved / ref["GBps"], 4)}
    mech = run_mechanisms(args, tin, tout, pool, torch, imgs, refs) if args.mechanisms else {}
    mech[args.callback] = {"jobs_per_s": round(set_jps, 1), "verified": bool(set_ok), "wrong_jobs": int(set_bad),
                           "steps": args.steps, "host_cpu_s_per_s": round(set_cpu, 2),
                           "host_us_per_job_launch": round(st.host_ns_launch / 1e3 / max(1, st.completed), 2)}

    # Each baseline runs with every copy mechanism and is scored by its
    # fastest, so SET's copy choice is not compared with a baseline held to
    # a worse one.
    extra = {}
    if not args.no_baselines and args.only is None:
        for mode in ("batch", "sync", "queue"):
            per = {}
            combos = [("kernels", 0), ("async_in", 0), ("nodes", 0)]
            if args.input_copy_streams > 0:
                combos.append(("async_in", args.input_copy_streams))
            for cp, cs in combos:
                key = cp if cs == 0 else "%s+%d_copy_streams" % (cp, cs)
                log("%s baseline, copy %s: %d jobs x %d steps" % (mode, key, args.jobs, args.baseline_steps))
                tout.zero_()
                c2, _, dt2, st2, (t2, _) = run_mode(mode, args, args.jobs, args.baseline_steps, 1, tin, tout, pool,
                                                    torch, copy=cp, copy_streams=cs)
                c2.close()
                ok2, bad2 = verify(tout, args.jobs, imgs, refs)
                lat2 = (t2["t_done"] - t2["t_launch"]) / 1e3  # launch (of the job, or of its batch) to completion
                per[key] = {"jobs_per_s": round(args.jobs * args.baseline_steps / dt2, 1), "verified": ok2,
                            "wrong_jobs": int(bad2), "host_sync_ms": round(st2.host_ns_sync / 1e6, 2),
                            "launch_to_done_p50_us": round(nearest_rank(lat2, 50), 1),
                            "launch_to_done_p99_us": round(nearest_rank(lat2, 99), 1)}
            best = max(per, key=lambda c: per[c]["jobs_per_s"])
            extra[mode] = {"jobs_per_s": per[best]["jobs_per_s"], "copy": best,
                           "launch_to_done_p50_us": per[best]["launch_to_done_p50_us"],
                           "launch_to_done_p99_us": per[best]["launch_to_done_p99_us"],
                           "verified": all(v["verified"] for v in per.values()), "by_copy": per}

    sections = {}
    if not args.no_sections:
        log("box/histogram jobs: 64")
        sections["box_hist_64"] = dict(box_section(args, torch), workload=(
            "64 jobs: 256x256 uint8 -> 3x3 box sum (zero-padded) -> floor(/9) -> 256-bin histogram, bit-exact; "
            "the plain method (sync launches, 4 streams), batch-sync (batch 8), the queue model and SET "
            "(4 workers x 4 slots)"))
        va = section_args(raw, "vectors")
        log("uneven vector jobs: %d" % va.vjobs)
        vout = vectors_section(va, torch)
        sections["vector_jobs"] = dict(vectors_summary(vout), modes=vout, workload=(
            "%d vector jobs, n log-uniform in [4096, 4194304), SAXPY -> tanh -> sum over device-resident pools" % va.vjobs),
            config={"workers": va.workers, "copy": va.copy, "callback": va.callback, "dispatchers": va.dispatchers,
                    "batch_max": va.batch_max, "tiles_max": va.tiles_max})
        torch.cuda.empty_cache()
        sa = section_args(raw, "scan")
        log("scan jobs: %d" % sa.scan_jobs)
        scpu = {}
        sruns = scan_section(sa, torch, [("set", 8, True, sa.copy), ("set", 8, False, sa.copy),
                                         ("batch", 8, False, "kernels"), ("batch", 8, False, "async_in"),
                                         ("queue", 8, False, "async_in")], scpu)
        sbest = max(r["jobs_per_s"] for r in sruns if r["mode"] == "set")
        sections["scan_jobs"] = dict(scan_summary(sruns), runs=sruns, cpu_oracle=scpu or None,
                                     pipeline_roofline={
                                         "bound": "host link, both directions",
                                         "achieved_GBps": round(sbest * (4 + 8) * (1 << 21) / 1e9, 2),
                                         "note": "8 MiB in + 16 MiB out per job; the link probe of this run gives "
                                                 "the host-to-device direction alone"},
                                     workload=(
            "%d jobs: 8 MiB int32 H2D -> inclusive int64 scan -> 16 MiB D2H, 8 workers" % sa.scan_jobs),
            config={"copy": sa.copy, "callback": sa.callback, "dispatchers": sa.dispatchers,
                    "inflight_per_worker": sa.inflight})
        torch.cuda.empty_cache()
        ga = section_args(raw, "serve", serve_seconds=args.section_serve_seconds, serve_pool=4)
        log("serving: %s requests/s, %.0f s windows" % (ga.rates, ga.serve_seconds))
        sres = serve_section(ga, torch)
        sections["serving"] = {"rates": sres, "verified": all(r["verified"] for r in sres), "workload": (
            "open-loop Poisson arrivals, 50%% images {256,512,1024,2048}^2 + 50%% vector jobs, %.0f GB admission cap, "
            "%.0f s window per rate" % (ga.mem_budget / 1e9, ga.serve_seconds)),
            "config": {"workers": ga.workers, "slots": ga.slots, "copy": ga.copy, "callback": ga.callback,
                       "dispatchers": ga.dispatchers, "inflight_per_worker": ga.inflight,
                       "image_pool_per_size": ga.serve_pool}}

    log("link probe")
    link_peak = link_probe(torch)
    # Scheduling-overhead fraction t_schedule / T_measured (Section 5.3, Eq. 4).
    # t_in is the input at the link's probed rate (several copies in flight
    # share the link at that rate; one copy alone on one stream is slower, and
    # is given beside it).  Two readings of T_ideal: Eq. 1 per batch of b jobs
    # (b = the workers or the batch size; 1 for the synchronous model), and the
    # link floor: every job's input back to back over the link, plus one job's
    # kernels and output copy.
    eq1["t_in_one_stream_us"] = eq1.pop("t_in_us")
    eq1["t_in_us"] = round(ib / (link_peak * 1e3), 3) if link_peak else eq1["t_in_one_stream_us"]

    def frac(jobs, T_s, b):
        per = eq1["t_k_us"] + eq1["t_out_us"]
        ideal = (jobs / b) * (b * eq1["t_in_us"] + per)
        floor = jobs * eq1["t_in_us"] + per
        T = T_s * 1e6
        return {"T_measured_ms": round(T / 1e3, 2), "eq1": round(1 - ideal / T, 4), "link_floor": round(1 - floor / T, 4)}
    overhead = {"terms": eq1, "set": frac(n_total, dt, args.workers)}
    for m, b_ in (("batch", args.batch), ("queue", args.workers), ("sync", 1)):
        if m in extra:
            overhead[m] = frac(args.jobs * args.baseline_steps, args.jobs * args.baseline_steps / extra[m]["jobs_per_s"], b_)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline(imgs, args.cpu_passes)

    h2d = ib * set_jps / 1e9
    per_step = [args.jobs / t for t in step_s]
    tl = traced
    tset = (tl or {}).get("modes", {}).get("set", {})
    line = {
        "metric": METRIC,
        "value": round(set_jps, 1),
        "unit": "jobs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gauss5-sobel-threshold-count/sum 1024x1024 f32 jobs, H2D 4 MiB + D2H 72 B each",
                   "jobs_per_step": args.jobs, "workers": args.workers, "slots_per_worker": args.slots,
                   "callback": args.callback, "dispatchers": args.dispatchers, "copy": args.copy,
                   "input_copy_streams": args.input_copy_streams, "inflight_per_worker": args.inflight,
                   "image_pool": pool},
        "verified": bool(set_ok),
        "wrong_jobs": int(set_bad),
        "h2d_GBps": round(h2d, 2),
        "batch_sync_jobs_per_s": extra.get("batch", {}).get("jobs_per_s"),
        "speedup_vs_batch_sync": round(set_jps / extra["batch"]["jobs_per_s"], 3) if "batch" in extra else None,
        "sync_jobs_per_s": extra.get("sync", {}).get("jobs_per_s"),
        "queue_jobs_per_s": extra.get("queue", {}).get("jobs_per_s"),
        "speedup_vs_queue": round(set_jps / extra["queue"]["jobs_per_s"], 3) if "queue" in extra else None,
        "speedup_vs_sync": round(set_jps / extra["sync"]["jobs_per_s"], 3) if "sync" in extra else None,
        "baselines": extra,
        "job_latency_us": {"launch_to_done_p50": round(nearest_rank(lat_dev, 50), 1),
                           "launch_to_done_p99": round(nearest_rank(lat_dev, 99), 1),
                           "submit_to_done_p50": round(nearest_rank(lat_sub, 50), 1),
                           "submit_to_done_p99": round(nearest_rank(lat_sub, 99), 1)},
        "steps_jobs_per_s": {"median": round(float(np.median(per_step)), 1), "min": round(float(min(per_step)), 1),
                             "max": round(float(max(per_step)), 1), "each": [round(float(v), 1) for v in per_step]},
        "pipeline_roofline": {"bound": "host-to-device link", "achieved_GBps": round(h2d, 2),
                              "peak_GBps": link_peak, "frac": round(h2d / link_peak, 4) if link_peak else None,
                              "peak_source": "hipMemcpyAsync of 64 MiB from pinned memory alone, best of 2 / 4 "
                                             "streams, 1 GiB each, measured in this run"},
        "sched": {"stolen": int(st.stolen), "inflight_high_water": int(st.inflight_high_water),
                  "host_us_per_job_bind": round(st.host_ns_bind / 1e3 / max(1, st.completed), 2),
                  "host_us_per_job_launch": round(st.host_ns_launch / 1e3 / max(1, st.completed), 2),
                  "host_us_per_job_callback": round(st.host_ns_callback / 1e3 / max(1, st.completed), 2)},
        # from the traced child runs of this invocation: gap on the timeline
        # with DMA copies counted as GPU work (the figure comparable across
        # copy mechanisms), kernels alone beside it
        "mean_kernel_gap_us": tset.get("mean_gap"),
        "mean_kernel_gap_kernels_only_us": tset.get("mean_kernel_gap"),
        "gpu_idle_fraction": tset.get("gpu_idle_fraction"),
        "timeline": tl,
        "overhead_fraction": overhead,
        "completion_mechanisms": mech,
        "configs": sections,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
