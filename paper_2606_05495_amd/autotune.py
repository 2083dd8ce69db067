"""Autotuner for the bucketed persistent vector batches.

Two levels.  For every size bucket b = floor(log2 n) present in a
calibration set, `tune` times each candidate (work-item size, persistent
grid) on that bucket's jobs through set_run_vector_jobs and keeps the
fastest.  `tune_blocks` runs that search once per candidate block size of the
work-item kernel (one template each: the block fixes the order in which an
item's elements are summed, so it is a property of the template, not of a
bucket) and keeps the block whose tuned buckets run the whole job set in the
least estimated time.  Results are cached as JSON keyed by (GPU
architecture, HIP runtime version): {"block": B, "buckets": {b: ...}}.

The candidate work-item sizes keep between 1 and 64 items per job; the grids
are multiples of the 256 compute units.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import _abi as A

TILES = (1024, 2048, 4096, 8192, 16384, 32768, 65536)
BLOCKS = (128, 256, 512, 1024)
GRIDS = (256, 512, 1024, 2048)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "vec_batch.json")


def _device_key():
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or p.name
    return "%s|hip-%s" % (arch.split(":")[0], torch.version.hip)


def bucket_of(n) -> np.ndarray:
    n = np.asarray(n, dtype=np.int64)
    return np.floor(np.log2(n)).astype(np.int64)


def candidates(b: int):
    lo, hi = 1 << b, (1 << (b + 1)) - 1
    for te in TILES:
        items_max = -(-hi // te)
        items_min = -(-lo // te)
        if items_max > 64 or (items_min < 1):
            continue
        if te > 4 * hi and te != TILES[0]:
            continue
        for g in GRIDS:
            yield te, g


def tuning_from(table: dict) -> A.set_vec_tuning:
    t = A.set_vec_tuning()
    for b, rec in table.items():
        t.tile_elems[int(b)] = int(rec["tile"])
        t.grid[int(b)] = int(rec["grid"])
    return t


def _record(cache):
    if not os.path.exists(cache):
        return None
    rec = json.load(open(cache)).get(_device_key())
    if rec and "buckets" not in rec:  # a table from before block sizes were tuned: block 256
        rec = {"block": 256, "buckets": rec}
    return rec


def load(cache: str = DEFAULT_CACHE):
    """The cached per-bucket tuning for this device, or None."""
    rec = _record(cache)
    return tuning_from(rec["buckets"]) if rec else None


def load_block(cache: str = DEFAULT_CACHE) -> int:
    """The cached block size of the work-item kernel for this device (0 = the library default)."""
    rec = _record(cache)
    return int(rec["block"]) if rec else 0


def _store(cache, rec):
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    db = json.load(open(cache)) if os.path.exists(cache) else {}
    db[_device_key()] = rec
    json.dump(db, open(cache, "w"), indent=1, sort_keys=True)


def tune_blocks(ctx, define, jobs: np.ndarray, calib: int = 512, reps: int = 3, cache: str = DEFAULT_CACHE,
                log=None):
    """define(block) -> template id of a vector batch template with that
    block.  Tunes every bucket for each block in BLOCKS and keeps the block
    whose best per-bucket times, scaled to the job set's bucket counts, add up
    to the least.  Returns (tuning, block) and caches both."""
    jobs = np.ascontiguousarray(jobs, dtype=A.VEC_JOB_DTYPE)
    bk = bucket_of(jobs["n"])
    counts = {int(b): int(np.sum(bk == b)) for b in set(bk.tolist())}
    best = None
    per_block = {}
    for blk in BLOCKS:
        tid = define(blk)
        table = _tune_table(ctx, tid, jobs, calib, reps, log)
        est = sum(rec["us"] * counts[int(b)] / rec["jobs"] for b, rec in table.items())
        per_block[blk] = round(est, 1)
        if log:
            log("block %d: estimated %.0f us for the %d jobs" % (blk, est, jobs.size))
        if best is None or est < best[0]:
            best = (est, blk, table)
    rec = {"block": best[1], "buckets": best[2], "estimated_us_by_block": per_block}
    if cache:
        _store(cache, rec)
    return tuning_from(best[2]), best[1]


def tune(ctx, tid: int, jobs: np.ndarray, calib: int = 512, reps: int = 3, cache: str = DEFAULT_CACHE,
         log=None) -> A.set_vec_tuning:
    """Time every candidate per bucket on up to `calib` jobs of that bucket
    (template tid, whose block stays as defined); store and return the table."""
    table = _tune_table(ctx, tid, jobs, calib, reps, log)
    if cache:
        _store(cache, {"block": int(ctx.templates[tid].block) if hasattr(ctx, "templates") else 0, "buckets": table})
    return tuning_from(table)


def _tune_table(ctx, tid: int, jobs: np.ndarray, calib: int, reps: int, log) -> dict:
    jobs = np.ascontiguousarray(jobs, dtype=A.VEC_JOB_DTYPE)
    bk = bucket_of(jobs["n"])
    table = {}
    for b in sorted(set(bk.tolist())):
        sel = jobs[bk == b][:calib]
        res = np.zeros(sel.size, np.float32)
        best = None
        for te, g in candidates(b):
            t = A.set_vec_tuning()
            t.tile_elems[b] = te
            t.grid[b] = g
            A.set_run_vector_jobs(ctx.h, tid, sel, res, t)  # warm
            dts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                A.set_run_vector_jobs(ctx.h, tid, sel, res, t)
                dts.append(time.perf_counter() - t0)
            dt = min(dts)
            if best is None or dt < best[0]:
                best = (dt, te, g)
        table[str(b)] = {"tile": best[1], "grid": best[2], "us": round(best[0] * 1e6, 1), "jobs": int(sel.size)}
        if log:
            log("bucket %d: tile %d grid %d  %.1f us for %d jobs" % (b, best[1], best[2], best[0] * 1e6, sel.size))
    return table
