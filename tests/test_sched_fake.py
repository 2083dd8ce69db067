"""Scheduler invariants (Algorithms 1-3) on the CPU fake backend: threads
stand in for streams, completions arrive on a separate callback thread.

Checked here without a GPU:
 (i)   every submitted id completes exactly once; ids are consecutive;
 (ii)  stealing happens only when enabled, and skewed submission forces it;
 (iii) a stolen job runs on the thief's slot (its output header says so);
 (iv)  no slot is used by two jobs at once (fake backend's in-use check +
       header canary flag);
 (v)   at most b*k jobs in flight;
 (vii) set_drain returns only when completed == submitted; timeouts and
       injected device errors surface as error codes.
"""
import os
import subprocess
import time
import threading

import numpy as np
import pytest

from paper_2606_05495_amd import _abi as A
from paper_2606_05495_amd.runtime import Context, out_header

DUMMY_POOL = (0x1000, 0x2000, 1 << 30)  # never dereferenced by the fake backend


def _vec_jobs(ctx, tid, n_jobs, dur_us, tags=None, hints=None):
    outs = np.zeros((n_jobs, 128), np.uint8)
    arr = ctx.job_array(n_jobs)
    arr["host_out"] = outs.ctypes.data + np.arange(n_jobs, dtype=np.uint64) * 128
    arr["out_bytes"] = 68
    arr["n"] = dur_us
    arr["a"] = 1.0
    arr["user_tag"] = np.arange(n_jobs) if tags is None else tags
    if hints is not None:
        arr["worker_hint"] = hints
    return arr, outs


def _headers(outs):
    return np.stack([out_header(outs[i]) for i in range(len(outs))])


def _fake(**kw):
    kw.setdefault("backend", "fake")
    return Context(**kw)


@pytest.mark.parametrize("b,d,nd", [(1, 2, 1), (4, 8, 1), (8, 16, 1), (8, 16, 4), (5, 4, 3), (2, 2, 8)])
def test_every_job_completes_once(b, d, nd):
    with _fake(workers=b, slots=d, dispatchers=nd) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 500, np.random.default_rng(0).integers(1, 60, 500))
        first = ctx.submit_many(tid, arr)
        assert first == 0
        ctx.drain()
        st = ctx.stats()
        assert st.submitted == st.completed == 500 and st.failed == 0
        h = _headers(outs)
        assert np.all(h["magic"] == A.SET_OUT_MAGIC)
        assert np.all(h["canary_ok"] == 1)
        assert np.array_equal(np.sort(h["job_id"]), np.arange(500))
        assert np.array_equal(h["user_tag"], np.arange(500))
        times = ctx.job_times()
        assert len(times) == 500 and len(set(times["job_id"].tolist())) == 500
        assert np.all(times["t_done"] >= times["t_launch"]) and np.all(times["t_launch"] >= times["t_submit"])
        assert st.inflight_high_water <= b * min(2, d)
        assert sum(st.launches_per_worker[:b]) == 500


@pytest.mark.parametrize("nd", [1, 2, 4])
def test_skewed_submission_forces_steals_and_retargets(nd):
    with _fake(workers=4, slots=8, submit_policy=A.SET_SUBMIT_SKEW0, dispatchers=nd) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 400, 200)
        ctx.submit_many(tid, arr)
        ctx.drain()
        st = ctx.stats()
        assert st.stolen > 0
        h = _headers(outs)
        t = ctx.job_times()
        by_id = {int(r["job_id"]): r for r in t}
        stolen_ids = [i for i, r in by_id.items() if r["stolen"]]
        assert len(stolen_ids) == st.stolen
        # a stolen job ran on its thief (worker != 0) and its header says so
        for i in stolen_ids:
            k = int(np.nonzero(h["job_id"] == i)[0][0])
            assert h["worker"][k] == by_id[i]["worker"] != 0
            assert h["slot"][k] == by_id[i]["slot"]
        assert np.all(h["canary_ok"] == 1)
        assert sum(st.launches_per_worker[1:4]) > 0


def test_256_workers_with_steals():
    """b up to 256 workers (the largest batch size the SET sweep runs): every job completes once,
    jobs skewed onto worker 0 are stolen by the others, and b = 257 is refused."""
    with _fake(workers=256, slots=2, submit_policy=A.SET_SUBMIT_SKEW0, dispatchers=4) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 600, 2000)
        ctx.submit_many(tid, arr)
        ctx.drain()
        st = ctx.stats()
        assert st.completed == 600 and st.failed == 0
        assert st.stolen > 0
        h = _headers(outs)
        assert np.array_equal(np.sort(h["job_id"]), np.arange(600))
        assert len(set(h["worker"].tolist())) > 1
    with pytest.raises(A.SetError):
        _fake(workers=257, slots=2)


@pytest.mark.parametrize("nd", [1, 3])
def test_no_stealing_keeps_jobs_local(nd):
    with _fake(workers=4, slots=8, submit_policy=A.SET_SUBMIT_SKEW0, stealing=False, dispatchers=nd) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 100, 50)
        ctx.submit_many(tid, arr)
        ctx.drain()
        st = ctx.stats()
        assert st.stolen == 0
        assert np.all(_headers(outs)["worker"] == 0)
        assert st.launches_per_worker[0] == 100


def test_worker_hint_and_local_first():
    with _fake(workers=3, slots=4) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 30, 10, hints=np.full(30, 2))
        ctx.submit_many(tid, arr)
        ctx.drain()
        h = _headers(outs)
        t = ctx.job_times()
        # jobs that were not stolen ran on the hinted worker
        for r in t:
            if not r["stolen"]:
                assert r["worker"] == 2


def _wait_until(pred, timeout_s=5.0):
    t0 = time.monotonic()
    while not pred():
        assert time.monotonic() - t0 < timeout_s, "setup did not reach the expected state"
        time.sleep(0.0005)


# Algorithm 2 (FindJob), C7 (ii): the thief's own queue is popped first; only
# when it is empty are victims probed, in the order (w+1), (w+2), ... (w+b-1)
# mod b, and the head of the first non-empty one is taken.
# (thief, workers whose queues get one job each, listed in submission order)
FINDJOB_SCENES = [
    (0, [3, 2, 1]),     # victims 1, 2, 3 in that order
    (2, [1, 0, 3]),     # wraps: 3, then 0, then 1 (a reversed probe would take 1 first)
    (1, [3, 1, 0, 2]),  # own queue first, then 2, 3, 0 (stealing before the local pop would take 2 first)
    (3, [2, 0]),        # 0 before 2 (from w+1 = 0 on)
]


@pytest.mark.parametrize("thief,filled", FINDJOB_SCENES)
def test_findjob_pops_local_then_probes_victims_in_order(thief, filled):
    """Four workers with one launch permit and one queue entry each.  Every
    worker first runs one job: the thief's ends after 0.15 s, the others' run
    0.9 s.  While all four run, one short job is queued on each worker of
    `filled`.  The only permit that comes back before 0.9 s is the thief's, so
    the thief takes every queued job, one after the other, and the order it
    takes them in is the order FindJob probes the queues: its own queue, then
    (w+1) ... (w+3) mod 4.  The setup is deterministic up to the 0.75 s margin."""
    with _fake(workers=4, slots=2, inflight=1, queue_capacity=1, dispatchers=1) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        outs = np.zeros((4 + len(filled), 128), np.uint8)

        def job(k, w, dur_us):
            return ctx.submit(tid, host_out=outs[k].ctypes.data, out_bytes=68, n=dur_us, a=1.0, user_tag=k,
                              worker_hint=w)

        for w in range(4):  # one running job per worker; each launches from its own queue
            job(w, w, 150_000 if w == thief else 900_000)
            _wait_until(lambda: ctx.stats().launches_per_worker[w] == 1)
        st = ctx.stats()
        assert st.stolen == 0 and st.inflight_high_water == 4
        t_fill = time.monotonic()
        ids = {job(4 + i, w, 1000): w for i, w in enumerate(filled)}
        assert time.monotonic() - t_fill < 0.1, "the queued jobs must be in place before the thief's permit returns"
        ctx.drain()
        rows = sorted((r for r in ctx.job_times() if int(r["job_id"]) in ids), key=lambda r: r["t_launch"])
        assert len(rows) == len(filled)
        assert all(int(r["worker"]) == thief for r in rows), "a queued job ran on a worker other than the thief"
        taken = [ids[int(r["job_id"])] for r in rows]
        expect = sorted(filled, key=lambda v: (v - thief) % 4)
        assert taken == expect, (taken, expect)
        assert [int(r["stolen"]) for r in rows] == [0 if v == thief else 1 for v in expect]
        assert ctx.stats().stolen == sum(v != thief for v in filled)
        h = _headers(outs)
        assert np.all(h["canary_ok"] == 1) and np.all(h["magic"] == A.SET_OUT_MAGIC)


@pytest.mark.parametrize("policy", ["any", "busy"])
def test_steal_policy_idle_victim(policy):
    """A fresh context: four workers, one permit each, all free, held by one
    dispatcher in worker order.  One job is submitted to worker 1.  The
    dispatcher's first permit is worker 0's; FindJob(0) finds Q_0 empty and
    probes Q_1.  As printed (SET_STEAL_ANY) it takes the job, though worker 1
    is idle; SET_STEAL_BUSY skips a victim holding a free permit, and worker 1
    runs its own job."""
    sp = A.SET_STEAL_ANY if policy == "any" else A.SET_STEAL_BUSY
    with _fake(workers=4, slots=2, inflight=1, dispatchers=1, steal_policy=sp) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        outs = np.zeros((1, 128), np.uint8)
        jid = ctx.submit(tid, host_out=outs[0].ctypes.data, out_bytes=68, n=1000, a=1.0, worker_hint=1)
        ctx.drain()
        r = [r for r in ctx.job_times() if int(r["job_id"]) == jid][0]
        if policy == "any":
            assert int(r["worker"]) == 0 and int(r["stolen"]) == 1 and ctx.stats().stolen == 1
        else:
            assert int(r["worker"]) == 1 and int(r["stolen"]) == 0 and ctx.stats().stolen == 0


@pytest.mark.parametrize("policy", ["any", "busy"])
def test_skewed_submission_steals_under_both_policies(policy):
    """Everything submitted to Q_0 with eight workers and eight dispatcher
    threads: both policies steal (worker 0 is busy), every job completes once
    with its own header."""
    sp = A.SET_STEAL_ANY if policy == "any" else A.SET_STEAL_BUSY
    with _fake(workers=8, slots=4, inflight=2, dispatchers=8, steal_policy=sp,
               submit_policy=A.SET_SUBMIT_SKEW0) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 400, 200)
        first = ctx.submit_many(tid, arr)
        ctx.drain(timeout_ns=int(30e9))
        hs = _headers(outs)
        assert np.array_equal(hs["job_id"], first + np.arange(400))
        assert np.all(hs["canary_ok"] == 1)
        st = ctx.stats()
        assert st.completed == 400 and st.stolen > 0


def test_findjob_without_stealing_leaves_other_queues():
    """With stealing off the thief's returned permit finds its own queue empty
    and takes nothing: the queued jobs wait for their own workers."""
    with _fake(workers=4, slots=2, inflight=1, queue_capacity=1, dispatchers=1, stealing=False) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        outs = np.zeros((7, 128), np.uint8)
        for w in range(4):
            ctx.submit(tid, host_out=outs[w].ctypes.data, out_bytes=68, n=20_000 if w == 0 else 300_000, a=1.0,
                       worker_hint=w)
            _wait_until(lambda: ctx.stats().launches_per_worker[w] == 1)
        ids = {ctx.submit(tid, host_out=outs[4 + i].ctypes.data, out_bytes=68, n=1000, a=1.0, worker_hint=w): w
               for i, w in enumerate([1, 2, 3])}
        ctx.drain()
        for r in ctx.job_times():
            if int(r["job_id"]) in ids:
                assert int(r["worker"]) == ids[int(r["job_id"])] and int(r["stolen"]) == 0
        assert ctx.stats().stolen == 0


def test_out_of_order_callbacks_keep_memory_safety():
    with _fake(workers=4, slots=4, fake_reorder=True) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 600, np.random.default_rng(1).integers(1, 40, 600))
        ctx.submit_many(tid, arr)
        ctx.drain()
        h = _headers(outs)
        assert np.all(h["canary_ok"] == 1)
        # a slot is released only after its job's completion is recorded, so per (worker, slot)
        # the next launch never precedes the previous job's completion stamp
        t = ctx.job_times()
        for key in {(int(r["worker"]), int(r["slot"])) for r in t}:
            rs = sorted((r for r in t if (r["worker"], r["slot"]) == key), key=lambda r: r["t_launch"])
            for a, b in zip(rs, rs[1:]):
                assert b["t_launch"] >= a["t_done"]
        assert ctx.stats().completed == 600


def test_concurrent_submitters_get_unique_consecutive_ids():
    with _fake(workers=4, slots=8) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        outs = np.zeros((4, 100, 128), np.uint8)
        ids = [[] for _ in range(4)]

        def producer(p):
            for i in range(100):
                ids[p].append(ctx.submit(tid, host_out=outs[p, i].ctypes.data, out_bytes=68, n=5, a=1.0,
                                         user_tag=p * 1000 + i))

        th = [threading.Thread(target=producer, args=(p,)) for p in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        ctx.drain()
        all_ids = sorted(sum(ids, []))
        assert all_ids == list(range(400))
        for p in range(4):
            assert ids[p] == sorted(ids[p])
            for i in range(100):
                h = out_header(outs[p, i])
                assert h["job_id"] == ids[p][i] and h["user_tag"] == p * 1000 + i


def test_drain_timeout_then_completion():
    with _fake(workers=1, slots=2) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 3, 300000)  # 0.3 s each
        ctx.submit_many(tid, arr)
        with pytest.raises(A.SetError) as e:
            ctx.drain(timeout_ns=1_000_000)
        assert e.value.code == A.SET_ETIMEOUT
        ctx.drain()
        assert ctx.stats().completed == 3


def test_nonblocking_submit_reports_full_staging():
    with _fake(workers=1, slots=2, staging=4) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        outs = np.zeros((64, 128), np.uint8)
        got = [ctx.submit(tid, host_out=outs[i].ctypes.data, out_bytes=68, n=20000, a=1.0, flags=A.SET_NONBLOCK)
               for i in range(64)]
        assert -1 in got  # SET_EAGAIN surfaced as -1
        accepted = [g for g in got if g >= 0]
        assert accepted == list(range(len(accepted)))
        ctx.drain()
        assert ctx.stats().completed == len(accepted)


def test_injected_device_error_latches_context():
    with _fake(workers=2, slots=4, fake_fail_after=5) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 40, 100)
        try:
            ctx.submit_many(tid, arr)
        except A.SetError as e:
            assert e.code == A.SET_EDEVICE
        with pytest.raises(A.SetError) as e:
            ctx.drain()
        assert e.value.code == A.SET_EDEVICE
        st = ctx.stats()
        assert st.completed == st.submitted and st.failed >= 1
        assert "injected" in A.set_last_error(ctx.h)
        with pytest.raises(A.SetError) as e2:
            ctx.submit(tid, host_out=outs[0].ctypes.data, out_bytes=68, n=5, a=1.0)
        assert e2.value.code == A.SET_EDEVICE


def test_memory_budget_bounds_bound_slots():
    with _fake(workers=4, slots=8) as ctx0:
        tid0 = ctx0.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        fp = A.set_template_footprint(ctx0.cfg, ctx0.templates[tid0])[0]
    with _fake(workers=4, slots=8, mem_budget=3 * fp) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 200, 100)
        ctx.submit_many(tid, arr)
        ctx.drain()
        st = ctx.stats()
        assert st.completed == 200
        assert 0 < st.mem_high_water <= 3 * fp
        assert st.inflight_high_water <= 3
        assert st.mem_in_use == 0


@pytest.mark.parametrize("mode", ["sync", "graph", "batch"])
def test_baseline_modes_complete_in_order(mode):
    with _fake(mode=mode, workers=4, slots=2) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 37, 30)
        ctx.submit_many(tid, arr)
        ctx.drain()
        st = ctx.stats()
        assert st.completed == 37 and st.stolen == 0
        h = _headers(outs)
        assert np.array_equal(h["job_id"], np.arange(37))
        assert np.all(h["worker"] == np.arange(37) % 4)
        if mode == "batch":
            assert st.batches == 10  # 9 full batches of 4 and one of 1 at drain


def test_batch_larger_than_worker_count_spans_slots():
    """A batch of more chains than workers: chain i runs in slot i // b of
    worker i % b, so batch_size may reach workers * slots and no more."""
    with _fake(mode="batch", workers=3, slots=4, batch_size=10) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 25, 30)
        ctx.submit_many(tid, arr)
        ctx.drain()
        st = ctx.stats()
        assert st.completed == 25 and st.batches == 3  # 10 + 10 + 5 at drain
        h = _headers(outs)
        assert np.array_equal(h["job_id"], np.arange(25))
        pos = np.arange(25) % 10  # chain index within its batch
        assert np.array_equal(h["worker"], pos % 3)
        assert np.array_equal(h["slot"], pos // 3)
    with pytest.raises(A.SetError):
        _fake(mode="batch", workers=3, slots=4, batch_size=13)


def test_invalid_arguments_rejected():
    with _fake(workers=2, slots=2) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1000, pool_ptrs=DUMMY_POOL)
        out = np.zeros(128, np.uint8)
        with pytest.raises(A.SetError) as e:
            ctx.submit(tid, host_out=out.ctypes.data, out_bytes=68, n=5000, a=1.0)  # n > max_n
        assert e.value.code == A.SET_EINVAL
        with pytest.raises(A.SetError):
            ctx.submit(tid + 5, host_out=out.ctypes.data, out_bytes=68, n=5, a=1.0)
        with pytest.raises(A.SetError):
            ctx.submit(tid, host_out=out.ctypes.data, out_bytes=8, n=5, a=1.0)  # output too small
        with pytest.raises(A.SetError):
            ctx.define("gauss_sobel", width=0, height=4)
    with pytest.raises(A.SetError):
        _fake(workers=0, slots=2)
    with pytest.raises(A.SetError):
        _fake(workers=2, slots=4, inflight=5)  # more permits than slots
    with pytest.raises(A.SetError):
        _fake(workers=2, slots=2, callback=A.SET_CB_EVENT_BLOCKING + 1)  # no such completion mechanism
    with pytest.raises(A.SetError):
        _fake(workers=2, slots=2, dispatchers=-1)
    for bad in (-1, 65):
        with pytest.raises(A.SetError):
            _fake(workers=2, slots=2, input_copy_streams=bad)
    _fake(workers=2, slots=2, input_copy_streams=64).close()  # capped at the worker count
    for cb in ("event_poll", "event_chain", "same_stream", "host_flag"):
        _fake(workers=2, slots=2, callback=cb).close()


def test_thread_sanitizer_stress():
    from paper_2606_05495_amd import build
    exe = build.build_tsan()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]


def test_thread_sanitizer_hip_backend_on_stub_runtime():
    """The HIP backend's own host code (backend_hip.hip compiled as C++) over a
    host-only runtime stand-in (csrc/hipstub: streams as in-order threads, a
    graph executable's parameters read when its nodes run and when it is
    launched), with the scheduler core, under ThreadSanitizer: every
    completion mechanism, up to 4 dispatcher threads, steals, DMA copies
    issued at bind, captured templates defined while jobs run, the comparison
    modes and vector batches.  No race report, every output header right, and
    no executable updated while a launch of it was queued or running."""
    from paper_2606_05495_amd import build
    exe = build.build_tsan_hip()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "0 executable updates overlapping" in r.stdout, r.stdout[-2000:]


# ------------------------------------------------------------------ bucketed persistent batching (host planning)
def _vec_job_array(ns, offs=0):
    jobs = np.zeros(len(ns), dtype=A.VEC_JOB_DTYPE)
    jobs["n"] = ns
    jobs["a"] = 1.0
    jobs["x_off"] = offs
    jobs["y_off"] = offs
    return jobs


def test_vector_batching_plans_buckets_and_limits():
    with _fake(workers=4, slots=4) as ctx:
        tid = ctx.define("saxpy_batch", max_n=1 << 22, pool_ptrs=DUMMY_POOL, batch_max=16, tiles_max=256)
        rng = np.random.default_rng(4)
        ns = np.floor(4096 * 1024.0 ** rng.random(300)).astype(np.int64)
        res, nb = ctx.run_vector_jobs(tid, _vec_job_array(ns))
        # expected plan: per bucket (floor log2 n) in input order, <= 16 jobs and <= 256 items per batch
        exp = 0
        for b in range(64):
            idx = [i for i, n in enumerate(ns) if int(n).bit_length() - 1 == b]
            if not idx:
                continue
            te = max(1024, min(65536, ((1 << max(b - 3, 0)) + 1023) // 1024 * 1024))
            cnt = tiles = 0
            exp += 1
            for i in idx:
                nt = -(-int(ns[i]) // te)
                if cnt >= 16 or tiles + nt > 256:
                    exp += 1
                    cnt = tiles = 0
                cnt += 1
                tiles += nt
        assert nb == exp
        st = ctx.stats()
        assert st.completed == nb and st.failed == 0


def test_vector_batching_rejects_bad_jobs_and_tuning():
    with _fake(workers=2, slots=2) as ctx:
        tid = ctx.define("saxpy_batch", max_n=1 << 20, pool_ptrs=DUMMY_POOL, batch_max=8, tiles_max=8)
        with pytest.raises(A.SetError):
            ctx.run_vector_jobs(tid, _vec_job_array([1 << 21]))  # n > max_n
        tune = A.set_vec_tuning()
        tune.tile_elems[12] = 1000  # not a multiple of 1024
        with pytest.raises(A.SetError):
            ctx.run_vector_jobs(tid, _vec_job_array([5000]), tuning=tune)
        tune.tile_elems[12] = 1024
        tune.tile_elems[19] = 1024  # 2^19-element job would need 512 items > tiles_max
        with pytest.raises(A.SetError):
            ctx.run_vector_jobs(tid, _vec_job_array([1 << 19]), tuning=tune)
        # one bucket; default 1024-element items: 4 + 5 + 8 items > tiles_max = 8 -> three batches
        res, nb = ctx.run_vector_jobs(tid, _vec_job_array([4096, 5000, 8191]), tuning=None)
        assert nb == 3


# ------------------------------------------------------------------ serving loop
def _serve_requests(ctx, t_img, t_vec, n_req, rate, seed=0, outs=None):
    from paper_2606_05495_amd import synth
    arr = synth.poisson_arrivals(seed, rate, n_req / rate * 2)[:n_req]
    req = np.zeros(len(arr), dtype=A.REQUEST_DTYPE)
    req["t_arrival_ns"] = (arr * 1e9).astype(np.uint64)
    kind = np.arange(len(arr)) % 2
    req["template_id"] = np.where(kind == 0, t_img, t_vec)
    req["worker_hint"] = -1
    outs = np.zeros((len(arr), 128), np.uint8) if outs is None else outs
    req["host_out"] = outs.ctypes.data + np.arange(len(arr), dtype=np.uint64) * 128
    req["out_bytes"] = 68
    req["n"] = np.where(kind == 0, 50, 4096 + 7 * np.arange(len(arr)))
    req["a"] = 1.0
    return req, outs


def test_serve_completes_every_request_and_batches_vectors():
    with _fake(workers=4, slots=4) as ctx:
        t_img = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        t_vec = ctx.define("saxpy_batch", max_n=1 << 20, pool_ptrs=DUMMY_POOL, batch_max=64, tiles_max=4096)
        req, outs = _serve_requests(ctx, t_img, t_vec, 400, rate=4000.0)
        vres = np.zeros(len(req), np.float32)
        cfg = A.set_serve_config()
        cfg.vec_inflight = 2
        done, st = A.set_serve(ctx.h, req, cfg, vres)
        assert st.arrived == len(req) and st.completed == len(req) and st.failed == 0 and st.not_admitted == 0
        assert np.all(done > 0) and np.all(done >= req["t_arrival_ns"])
        nvec = int(np.sum(req["template_id"] == t_vec))
        assert 1 <= st.vec_batches <= nvec  # vector requests were batched
        img = req["template_id"] == t_img
        for i in np.nonzero(img)[0][:50]:
            h = out_header(outs[i])
            assert h["magic"] == A.SET_OUT_MAGIC and h["canary_ok"] == 1


def test_serve_window_and_budget():
    with _fake(workers=2, slots=8) as ctx0:
        t0 = ctx0.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        fp = A.set_template_footprint(ctx0.cfg, ctx0.templates[t0])[0]
    with _fake(workers=2, slots=8, mem_budget=2 * fp) as ctx:
        t_img = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        t_vec = ctx.define("saxpy_batch", max_n=1 << 20, pool_ptrs=DUMMY_POOL, batch_max=16, tiles_max=1024)
        req, outs = _serve_requests(ctx, t_img, t_vec, 300, rate=3000.0, seed=3)
        cfg = A.set_serve_config()
        cfg.window_ns = int(req["t_arrival_ns"][150])
        done, st = A.set_serve(ctx.h, req, cfg, np.zeros(len(req), np.float32))
        assert st.arrived == 151 and st.not_admitted == len(req) - 151
        assert st.completed == 151
        assert np.all(done[:151] > 0) and np.all(done[151:] == 0)
        assert ctx.stats().mem_high_water <= 2 * fp


def test_queue_model_completes_and_spreads_work():
    with _fake(mode="queue", workers=4, slots=2) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 300, np.random.default_rng(2).integers(1, 50, 300))
        ctx.submit_many(tid, arr)
        ctx.drain()
        st = ctx.stats()
        assert st.completed == 300 and st.stolen == 0 and st.failed == 0
        h = _headers(outs)
        assert np.all(h["magic"] == A.SET_OUT_MAGIC) and np.all(h["canary_ok"] == 1)
        assert np.array_equal(np.sort(h["job_id"]), np.arange(300))
        assert all(st.launches_per_worker[w] > 0 for w in range(4))
        assert np.all(h["slot"] == 0)


def test_define_template_while_other_jobs_run():
    """A template defined while jobs of another template are in flight (storage never moves under them)."""
    import threading
    with _fake(workers=4, slots=4, dispatchers=2) as ctx:
        t0 = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr0, outs0 = _vec_jobs(ctx, t0, 600, 20)
        th = threading.Thread(target=lambda: ctx.submit_many(t0, arr0))
        th.start()
        tids = [ctx.define("saxpy_tanh_sum", max_n=1 << 18, pool_ptrs=DUMMY_POOL) for _ in range(6)]
        th.join()
        arrs = [_vec_jobs(ctx, t, 50, 10) for t in tids]
        for t, (arr, _) in zip(tids, arrs):
            ctx.submit_many(t, arr)
        ctx.drain()
        st = ctx.stats()
        assert st.completed == 600 + 6 * 50 and st.failed == 0
        assert np.all(_headers(outs0)["magic"] == A.SET_OUT_MAGIC)
        for _, outs in arrs:
            assert np.all(_headers(outs)["canary_ok"] == 1)


def test_library_scan_template_rules():
    """Library-call templates: fixed length (n = max_n), no low-word output, no batch graph."""
    with _fake(workers=2, slots=2) as ctx:
        tid = ctx.define("scan_lib", max_n=1000)
        assert ctx.out_bytes(tid) == 64 + 8 * 1000 and ctx.in_bytes(tid) == 4 * 1000
        names = [n for n, _ in ctx.stage_info(tid)]
        assert names == ["job_begin", "scan_lib_rocprim", "job_end"]
        inp = np.zeros(1000, np.int32)
        out = np.zeros(64 + 8 * 1000, np.uint8)
        with pytest.raises(A.SetError) as e:
            ctx.submit(tid, host_in=inp.ctypes.data, in_bytes=4 * 500, host_out=out.ctypes.data,
                       out_bytes=out.size, n=500)
        assert e.value.code == A.SET_EINVAL
        with pytest.raises(A.SetError):
            ctx.define("scan_lib", max_n=1000, flags=A.SET_TF_SCAN_LOW32)
    with _fake(mode="batch", workers=2, slots=1, batch_size=2) as ctx:
        with pytest.raises(A.SetError) as e:
            ctx.define("scan_lib", max_n=1000)
        assert e.value.code == A.SET_EUNSUPPORTED


def test_block_size_only_for_vector_batches():
    """set_job_template.block: 128/256/512/1024 (or 0) for the vector batch
    template, and 0 for every other pipeline."""
    with _fake(workers=2, slots=2) as ctx:
        for blk in (0, 128, 256, 512, 1024):
            ctx.define("saxpy_batch", max_n=1 << 20, pool_ptrs=DUMMY_POOL, batch_max=4, tiles_max=64, block=blk)
        for blk in (64, 100, 2048, -1):
            with pytest.raises(A.SetError):
                ctx.define("saxpy_batch", max_n=1 << 20, pool_ptrs=DUMMY_POOL, batch_max=4, tiles_max=64, block=blk)
        with pytest.raises(A.SetError):
            ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL, block=256)


def test_stress_template_options():
    """The memory-safety stress options: the poison flag and a delay of
    0..100000 us are accepted, a larger delay or a nonzero reserved field is
    refused.  On the fake backend the delay lengthens every job, and with one
    slot per worker under skewed submission no job runs in a slot another job
    still holds (the fake backend's clash check, reported per job as the
    canary flag)."""
    with _fake(workers=4, slots=1, submit_policy=A.SET_SUBMIT_SKEW0, dispatchers=2) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL, flags=A.SET_TF_POISON,
                         stress_delay_us=2000)
        ctx.define("gauss_sobel", width=8, height=8, flags=A.SET_TF_POISON, stress_delay_us=100000)
        with pytest.raises(A.SetError):
            ctx.define("gauss_sobel", width=8, height=8, stress_delay_us=100001)
        t = A.set_job_template()
        t.pipeline = A.SET_PIPE_GAUSS_SOBEL_F32
        t.width = t.height = 8
        t.reserved = 1
        with pytest.raises(A.SetError):
            A.set_template_define(ctx.h, t)
        arr, outs = _vec_jobs(ctx, tid, 16, 10)
        t0 = time.perf_counter()
        first = ctx.submit_many(tid, arr)
        ctx.drain(timeout_ns=int(10e9))
        dt = time.perf_counter() - t0
        hs = _headers(outs)
        assert np.all(hs["canary_ok"] == 1)
        assert np.array_equal(hs["job_id"], first + np.arange(16))
        assert dt >= 16 * 2010e-6 / 4  # four workers, each job at least 2 ms
        assert ctx.stats().stolen > 0


def test_device_copy_reference_needs_a_device():
    """set_time_device_copy: the fake backend has no device (SET_EUNSUPPORTED,
    the context stays usable); sizes outside 32 .. 2^30 bytes are refused."""
    with _fake(workers=2, slots=2) as ctx:
        with pytest.raises(A.SetError) as e:
            ctx.time_device_copy(1 << 20, 10)
        assert e.value.code == A.SET_EUNSUPPORTED
        for nbytes, reps in ((16, 10), ((1 << 30) + 1, 10), (1 << 20, 0)):
            with pytest.raises(A.SetError):
                ctx.time_device_copy(nbytes, reps)
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        arr, outs = _vec_jobs(ctx, tid, 4, 10)
        ctx.submit_many(tid, arr)
        ctx.drain(timeout_ns=int(5e9))
        assert ctx.stats().completed == 4


def test_empty_inputs():
    """Empty submissions and empty vector batches are no-ops: nothing is
    counted, drain returns at once, and the context stays usable."""
    with _fake(workers=2, slots=2) as ctx:
        tid = ctx.define("saxpy_tanh_sum", max_n=1 << 20, pool_ptrs=DUMMY_POOL)
        tb = ctx.define("saxpy_batch", max_n=1 << 20, pool_ptrs=DUMMY_POOL, batch_max=4, tiles_max=64)
        ctx.submit_many(tid, ctx.job_array(0))
        ctx.drain(timeout_ns=int(1e9))
        res, nb = ctx.run_vector_jobs(tb, np.zeros(0, dtype=A.VEC_JOB_DTYPE))
        assert nb == 0 and res.size == 0
        st = ctx.stats()
        assert st.submitted == 0 and st.completed == 0
        arr, outs = _vec_jobs(ctx, tid, 3, 10)
        assert ctx.submit_many(tid, arr) == 0
        ctx.drain()
        assert ctx.stats().completed == 3
