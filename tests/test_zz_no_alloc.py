"""The no-allocation vector-sum call against set_run_vector_jobs.

set_run_vector_jobs_noalloc keeps its work area in a static device array and
allocates nothing; for the same jobs and item sizes each job's S must be
bit-identical to set_run_vector_jobs's (both sum a job's item partials in item
order, and an item's partial depends only on its elements).  Two calls in a
row, the second smaller, so a stale table, counter or partial left by the
first call would show.  Also pinned to the oracle within its tolerance.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2606_05495_amd import _abi as A
from paper_2606_05495_amd import synth
from paper_2606_05495_amd.runtime import Context

pytestmark = pytest.mark.gpu

POOL = 1 << 23


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def pools(torch_gpu):
    x = synth.vec_pool(0, "x", POOL)
    y = synth.vec_pool(0, "y", POOL)
    return x, y, torch_gpu.from_numpy(x).cuda(), torch_gpu.from_numpy(y).cuda()


def _jobs(seed, count, max_n):
    """Log-uniform lengths in [1, max_n], windows at every alignment mod 4."""
    rng = np.random.default_rng(seed)
    n = np.floor(np.exp(rng.uniform(0, np.log(max_n + 1), count))).astype(np.int64)
    n = np.clip(n, 1, max_n)
    jobs = np.zeros(count, dtype=A.VEC_JOB_DTYPE)
    jobs["n"] = n
    jobs["a"] = (0.5 + 1.5 * rng.random(count)).astype(np.float32)
    jobs["x_off"] = rng.integers(0, POOL - n + 1)
    jobs["y_off"] = rng.integers(0, POOL - n + 1)
    return jobs


def _noalloc(torch, xd, yd, jobs, max_n, tuning=None, grid=0):
    jd = torch.from_numpy(jobs.view(np.uint8).copy()).cuda()
    rd = torch.full((len(jobs),), -7.0, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    A.set_run_vector_jobs_noalloc(torch.cuda.current_device(), st.cuda_stream, xd.data_ptr(), yd.data_ptr(),
                                  min(xd.numel(), yd.numel()), max_n, jd.data_ptr(), len(jobs), rd.data_ptr(),
                                  tuning, grid)
    st.synchronize()
    return rd.cpu().numpy()


def _batched(xd, yd, jobs, max_n, tuning=None):
    ctx = Context(mode="set", workers=2, slots=4)
    try:
        tid = ctx.define("saxpy_batch", max_n=max_n, x_pool=xd, y_pool=yd, batch_max=1024, tiles_max=1 << 16)
        res, _ = ctx.run_vector_jobs(tid, jobs, tuning=tuning)
    finally:
        ctx.close()
    return res


@pytest.mark.parametrize("tiles", ["default", "tuned"])
def test_noalloc_matches_batched_two_calls(torch_gpu, pools, tiles):
    x, y, xd, yd = pools
    max_n = 1 << 22
    tune = None
    if tiles == "tuned":
        # half the default item size below bucket 21 (at most 64 items a job)
        tune = A.set_vec_tuning()
        for b in range(64):
            default = min(65536, max(1024, -(-(1 << max(b - 3, 0)) // 1024) * 1024))
            tune.tile_elems[b] = default if b >= 21 else max(1024, default // 2048 * 1024)
    for call, (seed, count) in enumerate(((11, 3000), (12, 700))):
        _say("noalloc", tiles, "call", call, "jobs", count)
        jobs = _jobs(seed + (tiles == "tuned"), count, max_n)
        got = _noalloc(torch_gpu, xd, yd, jobs, max_n, tune, grid=0 if call == 0 else 300)
        ref = _batched(xd, yd, jobs, max_n, tune)
        bad = np.nonzero(got.view(np.uint32) != ref.view(np.uint32))[0]
        assert bad.size == 0, (call, bad[:5], got[bad[:5]], ref[bad[:5]])
        for i in range(0, count, 97):
            n, xo, yo = int(jobs["n"][i]), int(jobs["x_off"][i]), int(jobs["y_off"][i])
            S, E = oracle.saxpy_tanh_sum(x[xo:xo + n], y[yo:yo + n], jobs["a"][i])
            assert abs(float(got[i]) - S) <= oracle.vec_tolerance(S, E), (i, n, got[i], S)


def test_noalloc_rejected_jobs_and_limits(torch_gpu, pools):
    """Jobs outside [1, max_n] or leaving a pool give NaN and leave the others
    exact; counts above the stated maximum are refused on the host."""
    x, y, xd, yd = pools
    max_n = 1 << 16
    jobs = _jobs(5, 40, max_n)
    jobs["n"][3] = 0
    jobs["n"][7] = max_n + 1
    jobs["x_off"][11] = POOL - 10
    jobs["n"][11] = 11
    got = _noalloc(torch_gpu, xd, yd, jobs, max_n)
    assert np.isnan(got[[3, 7, 11]]).all()
    keep = np.setdiff1d(np.arange(40), [3, 7, 11])
    ref = _batched(xd, yd, jobs[keep], max_n)
    assert np.array_equal(got[keep].view(np.uint32), ref.view(np.uint32))
    with pytest.raises(A.SetError) as e:
        A.set_run_vector_jobs_noalloc(0, 0, xd.data_ptr(), yd.data_ptr(), POOL, max_n, xd.data_ptr(),
                                      A.SET_NOALLOC_MAX_JOBS + 1, yd.data_ptr())
    assert e.value.code == A.SET_EINVAL and "16384" in str(e.value)
