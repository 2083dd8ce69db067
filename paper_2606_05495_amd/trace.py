"""Timeline metrics from rocprofv3 traces (kernel-trace and memory-copy-trace CSVs).

Definitions (the paper gives prose definitions; these are the readings):

* kernel gap -- idle time between the end of one kernel and the start of the
  next on the GPU timeline (Section 1, the white spaces of a profiler
  timeline).  Kernels of all streams are merged by start time; gap_k =
  max(0, start_{k+1} - max_{i<=k} end_i).  The headline is the mean over all
  k (zeros included); the mean of the positive gaps is reported beside it.
  The same gap taken over kernels and DMA copies merged (mean_gap) counts a
  running copy as GPU work; it equals the kernel gap when every copy is a
  kernel, and it is the figure comparable across copy mechanisms.
* GPU-idle fraction -- 1 - |union of kernel and copy intervals| / span, the
  reading of the scheduling-overhead fraction t_schedule / T_measured
  (Section 5.3 with Eq. 4): T_measured is the span of the timeline and
  T_ideal the time some engine was busy, so t_schedule = T_measured - T_ideal.
  Compute-idle uses kernels only, copy-idle the host-to-device copies only
  (DMA copies and k_copy_in kernels).  The copy overlap fraction is the time
  both directions are busy over the time either is.
* inter-batch overhead (Eq. 3) -- for a batch-synchronised run, the start of
  batch i+1's first copy minus the end of batch i's last copy.

    python -m paper_2606_05495_amd.trace <dir with *_kernel_trace.csv>
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys
from typing import Iterable, List, Sequence, Tuple

Interval = Tuple[float, float]


def union_length(intervals: Iterable[Interval]) -> float:
    iv = sorted((a, b) for a, b in intervals if b > a)
    total = 0.0
    cur_a = cur_b = None
    for a, b in iv:
        if cur_b is None or a > cur_b:
            if cur_b is not None:
                total += cur_b - cur_a
            cur_a, cur_b = a, b
        else:
            cur_b = max(cur_b, b)
    if cur_b is not None:
        total += cur_b - cur_a
    return total


def merged(intervals: Iterable[Interval]) -> List[Interval]:
    """Disjoint, sorted union of the intervals."""
    out: List[Interval] = []
    for a, b in sorted((a, b) for a, b in intervals if b > a):
        if out and a <= out[-1][1]:
            out[-1] = (out[-1][0], max(out[-1][1], b))
        else:
            out.append((a, b))
    return out


def overlap_length(x: Iterable[Interval], y: Iterable[Interval]) -> float:
    """|union(x) intersect union(y)|."""
    mx, my = merged(x), merged(y)
    i = j = 0
    total = 0.0
    while i < len(mx) and j < len(my):
        lo, hi = max(mx[i][0], my[j][0]), min(mx[i][1], my[j][1])
        if hi > lo:
            total += hi - lo
        if mx[i][1] < my[j][1]:
            i += 1
        else:
            j += 1
    return total


def kernel_gaps(kernels: Sequence[Interval]) -> List[float]:
    ks = sorted(kernels)
    gaps = []
    end_max = None
    for i, (a, b) in enumerate(ks):
        if i > 0:
            gaps.append(max(0.0, a - end_max))
        end_max = b if end_max is None else max(end_max, b)
    return gaps


def timeline_metrics(kernels: Sequence[Interval], copies_h2d: Sequence[Interval] = (),
                     copies_d2h: Sequence[Interval] = ()) -> dict:
    """All times in one unit (the caller's); returns the metrics in that unit."""
    allv = list(kernels) + list(copies_h2d) + list(copies_d2h)
    if not allv:
        return {}
    t0 = min(a for a, _ in allv)
    t1 = max(b for _, b in allv)
    span = t1 - t0
    busy = union_length(allv)
    gaps = kernel_gaps(kernels)
    pos = [g for g in gaps if g > 0]
    ogaps = kernel_gaps(allv)
    out = {
        "mean_gap": (sum(ogaps) / len(ogaps)) if ogaps else 0.0,
        "span": span,
        "busy": busy,
        "gpu_idle_fraction": (1.0 - busy / span) if span > 0 else 0.0,
        "t_schedule": span - busy,
        "kernels": len(kernels),
        "mean_kernel_gap": (sum(gaps) / len(gaps)) if gaps else 0.0,
        "mean_positive_kernel_gap": (sum(pos) / len(pos)) if pos else 0.0,
        "compute_idle_fraction": (1.0 - union_length(kernels) / span) if span > 0 and kernels else None,
        "h2d_idle_fraction": (1.0 - union_length(copies_h2d) / span) if span > 0 and copies_h2d else None,
        "d2h_idle_fraction": (1.0 - union_length(copies_d2h) / span) if span > 0 and copies_d2h else None,
    }
    return out


def stream_gaps(kernels: Sequence[Interval], streams: Sequence, names: Sequence[str] = (),
                is_copy=lambda n: "copy" in n.lower(), is_tail=lambda n: "done_flag" in n) -> dict:
    """Gaps between consecutive kernels of the same stream.

    On one stream a job's kernels run in order (host-to-device copy, stages,
    device-to-host copy, optionally a completion-word kernel), so a gap there
    is dispatch latency: either between two kernels of one job (dependency
    resolution inside a graph) or between one job's last kernel and the next
    job's first copy (the launch path).  A copy that follows a copy or a
    completion-word kernel starts a new job; every other pair is a gap inside
    a job."""
    by = {}
    for i, (iv, s) in enumerate(zip(kernels, streams)):
        by.setdefault(s, []).append((iv[0], iv[1], names[i] if names else ""))
    allg, intra, inter = [], [], []
    for s, ks in by.items():
        ks.sort()
        for (a0, a1, an), (b0, b1, bn) in zip(ks, ks[1:]):
            g = max(0.0, b0 - a1)
            allg.append(g)
            if names and is_copy(bn) and (is_copy(an) or is_tail(an)):
                inter.append(g)
            else:
                intra.append(g)
    mean = lambda v: (sum(v) / len(v)) if v else None
    return {"streams": len(by), "mean_stream_gap": mean(allg), "mean_intra_job_gap": mean(intra),
            "mean_job_boundary_gap": mean(inter) if names else None}


def eq_terms(kernels: Sequence[Interval], streams: Sequence, names: Sequence[str],
             is_copy=lambda n: "copy" in n.lower(), is_tail=lambda n: "done_flag" in n) -> dict:
    """Per-job terms of the overhead model (Section 3.1, Eq. 1-2) from one
    stream's kernel sequence [input copy, stages..., output copy (, completion
    word)]: t_in, t_k (sum of stage durations), t_out, and the gaps t_in-k
    (input copy end to first stage), Delta t_k (between stages) and t_k-out
    (last stage to output copy).  Segments without that shape, or whose stage
    count differs from the most common one (chains interleaved on one
    stream), are skipped; `jobs` counts the ones used.  Means in the input's
    time unit."""
    by = {}
    for iv, s, n in zip(kernels, streams, names):
        by.setdefault(s, []).append((iv[0], iv[1], n))
    cands = []
    for ks in by.values():
        ks.sort()
        seg = []
        for a, b, n in ks + [(None, None, "")]:
            starts_job = n == "" or (is_copy(n) and (not seg or is_copy(seg[-1][2]) or is_tail(seg[-1][2])))
            if starts_job and seg:
                body = [x for x in seg if not is_tail(x[2])]
                if len(body) >= 3 and is_copy(body[0][2]) and is_copy(body[-1][2]) and \
                        not any(is_copy(x[2]) for x in body[1:-1]):
                    cands.append(body)
                seg = []
            if n:
                seg.append((a, b, n))
    acc = {"t_in": 0.0, "t_k": 0.0, "t_out": 0.0, "t_in_k": 0.0, "delta_t_k": 0.0, "t_k_out": 0.0}
    jobs = 0
    if cands:
        counts = {}
        for body in cands:
            counts[len(body)] = counts.get(len(body), 0) + 1
        m = max(counts, key=lambda k: (counts[k], -k))
        for body in cands:
            if len(body) != m:
                continue
            st = body[1:-1]
            acc["t_in"] += body[0][1] - body[0][0]
            acc["t_out"] += body[-1][1] - body[-1][0]
            acc["t_k"] += sum(b1 - a1 for a1, b1, _ in st)
            acc["t_in_k"] += max(0.0, st[0][0] - body[0][1])
            acc["t_k_out"] += max(0.0, body[-1][0] - st[-1][1])
            acc["delta_t_k"] += sum(max(0.0, st[i + 1][0] - st[i][1]) for i in range(len(st) - 1))
            jobs += 1
    out = {k: (v / jobs if jobs else None) for k, v in acc.items()}
    out["jobs"] = jobs
    return out


def inter_batch_gaps(h2d: Sequence[Interval], d2h: Sequence[Interval], batch: int) -> List[float]:
    """Eq. 3 for consecutive batches of `batch` jobs (copies in time order)."""
    hs = sorted(h2d)
    ds = sorted(d2h, key=lambda x: x[1])
    nb = min(len(hs), len(ds)) // batch
    starts = [hs[i * batch][0] for i in range(nb)]
    ends = [ds[(i + 1) * batch - 1][1] for i in range(nb)]
    return [starts[i + 1] - ends[i] for i in range(nb - 1)]


# ------------------------------------------------------------------ rocprofv3 CSV
def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(names)


def load_rocprof(dirpath: str, kernel_filter=None, copy_streams=None):
    """Kernel and copy intervals (ns) from rocprofv3 --kernel-trace
    --memory-copy-trace --output-format csv output under dirpath.  If
    copy_streams is a dict, it receives the stream of every DMA copy
    ({"h2d": [...], "d2h": [...]}, in the order of the returned intervals)."""
    kfiles = glob.glob(os.path.join(dirpath, "**", "*kernel_trace.csv"), recursive=True)
    cfiles = glob.glob(os.path.join(dirpath, "**", "*memory_copy_trace.csv"), recursive=True)
    kernels, names, streams = [], [], []
    for f in kfiles:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                name = _col(row, "Kernel_Name", "Kernel_name", "KernelName")
                if kernel_filter and not kernel_filter(name):
                    continue
                kernels.append((float(_col(row, "Start_Timestamp", "BeginNs")),
                                float(_col(row, "End_Timestamp", "EndNs"))))
                names.append(name)
                streams.append(row.get("Stream_Id") or row.get("Queue_Id") or "0")
    h2d, d2h = [], []
    cs = {"h2d": [], "d2h": []}
    for f in cfiles:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                d = _col(row, "Direction", "Kind", "Operation")
                iv = (float(_col(row, "Start_Timestamp", "BeginNs")), float(_col(row, "End_Timestamp", "EndNs")))
                sid = row.get("Stream_Id") or "0"
                if "HOST_TO_DEVICE" in d.upper() or "H2D" in d.upper():
                    h2d.append(iv)
                    cs["h2d"].append(sid)
                elif "DEVICE_TO_HOST" in d.upper() or "D2H" in d.upper():
                    d2h.append(iv)
                    cs["d2h"].append(sid)
    if copy_streams is not None:
        copy_streams.update(cs)
    return kernels, names, h2d, d2h, streams


def _clip(intervals, keep, t0, t1):
    """Intervals overlapping [t0, t1], clipped to it, with the parallel lists
    in `keep` filtered alike."""
    idx = [i for i, (a, b) in enumerate(intervals) if b > t0 and a < t1]
    return ([(max(intervals[i][0], t0), min(intervals[i][1], t1)) for i in idx],
            [[lst[i] for i in idx] for lst in keep])


def analyze_dir(dirpath: str, batch: int = 0, library_window: bool = False) -> dict:
    """Timeline metrics of a rocprofv3 trace directory.  library_window: the
    span runs from the first to the last of the library's own kernels only,
    and every other kernel or copy is clipped to it (for programs whose set-up
    uploads or host-side work come before the jobs)."""
    cs = {}
    kernels, names, h2d, d2h, streams = load_rocprof(
        dirpath, kernel_filter=lambda n: "setrt" in n or "copyBuffer" in n, copy_streams=cs)
    if library_window:
        lib = [iv for iv, n in zip(kernels, names) if "setrt" in n]
        if lib:
            t0, t1 = min(a for a, _ in lib), max(b for _, b in lib)
            kernels, (names, streams) = _clip(kernels, [names, streams], t0, t1)
            h2d, (cs["h2d"],) = _clip(h2d, [cs.get("h2d", [])], t0, t1)
            d2h, (cs["d2h"],) = _clip(d2h, [cs.get("d2h", [])], t0, t1)
    m = timeline_metrics(kernels, h2d, d2h)
    # DMA copies join their stream's sequence (as "dma_copy_*"), so a job whose
    # input went by DMA still reads as [input copy, stages, output copy]; the
    # kernel gap above stays over kernels only.
    ev = kernels + h2d + d2h
    ev_streams = streams + cs.get("h2d", []) + cs.get("d2h", [])
    ev_names = names + ["dma_copy_h2d"] * len(h2d) + ["dma_copy_d2h"] * len(d2h)
    m.update(stream_gaps(ev, ev_streams, ev_names))
    m["eq_terms"] = {k: (v / 1e3 if (v is not None and k != "jobs") else v)
                     for k, v in eq_terms(ev, ev_streams, ev_names).items()}
    us_keys = ("span", "busy", "t_schedule", "mean_gap", "mean_kernel_gap", "mean_positive_kernel_gap", "mean_stream_gap",
               "mean_intra_job_gap", "mean_job_boundary_gap")
    m = {k: (v / 1e3 if k in us_keys and v is not None else v) for k, v in m.items()}  # ns -> us
    m["unit"] = "us"
    m["h2d_copies"] = len(h2d)
    m["d2h_copies"] = len(d2h)
    # input and output copies of either kind: DMA copies and the copy kernels
    # (k_copy_in host-to-device, k_copy_out device-to-host)
    cin = h2d + [iv for iv, n in zip(kernels, names) if "k_copy_in" in n]
    cout = d2h + [iv for iv, n in zip(kernels, names) if "k_copy_out" in n]
    span = m.get("span") or 0.0
    if cin and span > 0:
        m["h2d_idle_fraction"] = 1.0 - union_length(cin) / (span * 1e3)
    if cin and cout:
        # both directions on the link at once, as a share of the time either is
        m["h2d_d2h_overlap_fraction"] = overlap_length(cin, cout) / union_length(cin + cout)
    if batch and cin and cout:
        g = inter_batch_gaps(cin, cout, batch)
        m["mean_inter_batch_us"] = (sum(g) / len(g) / 1e3) if g else None
    return m


def kernel_stats(dirpath: str) -> dict:
    """Per-kernel summary of a rocprofv3 --stats run (*_kernel_stats.csv)."""
    out = {}
    for f in glob.glob(os.path.join(dirpath, "**", "*kernel_stats.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                out[row["Name"]] = {"calls": int(row["Calls"]), "avg_us": float(row["AverageNs"]) / 1e3,
                                    "min_us": float(row["MinNs"]) / 1e3, "max_us": float(row["MaxNs"]) / 1e3,
                                    "total_ms": float(row["TotalDurationNs"]) / 1e6}
    return out


def isolated_run(dirpath: str, name_part: str) -> dict:
    """The longest run of back-to-back dispatches of one kernel on one stream
    with no other kernel of that stream in between (the stage-timing loop),
    and their mean duration (first dispatch of the run excluded)."""
    rows = []
    for f in glob.glob(os.path.join(dirpath, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                rows.append((row.get("Stream_Id") or row.get("Queue_Id") or "0",
                             float(_col(row, "Start_Timestamp", "BeginNs")), float(_col(row, "End_Timestamp", "EndNs")),
                             _col(row, "Kernel_Name", "Kernel_name", "KernelName")))
    rows.sort()
    best, cur = [], []
    prev_stream = None
    for stream, a, b, name in rows:
        if name_part in name and stream == prev_stream and cur:
            cur.append((a, b))
        elif name_part in name:
            cur = [(a, b)]
        else:
            cur = []
        prev_stream = stream
        if len(cur) > len(best):
            best = list(cur)
    if len(best) < 2:
        return {"dispatches": len(best)}
    d = [b - a for a, b in best[1:]]
    return {"dispatches": len(best) - 1, "avg_us": sum(d) / len(d) / 1e3,
            "wall_per_dispatch_us": (best[-1][1] - best[1][0]) / (len(best) - 1) / 1e3}


def pmc_values(dirpath: str, counter: str):
    """Per-dispatch values of one counter from a rocprofv3 --pmc run
    (*counter_collection.csv): [(dispatch_id, kernel_name, value)] in dispatch
    order, summed over the rows of a dispatch (one per agent block or XCD)."""
    acc = {}
    for f in glob.glob(os.path.join(dirpath, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if _col(row, "Counter_Name") != counter:
                    continue
                did = int(_col(row, "Dispatch_Id", "Correlation_Id"))
                name = _col(row, "Kernel_Name", "Kernel_name")
                v = float(_col(row, "Counter_Value"))
                prev = acc.get(did, (name, 0.0))
                acc[did] = (name, prev[1] + v)
    return [(d, n, v) for d, (n, v) in sorted(acc.items())]


def loop_average(values, name_part: str, last: int):
    """Mean counter value over the last `last` dispatches of the kernel whose
    name contains name_part (a cold loop's timed launches, which come after
    the batch's dispatches, the untimed passes and the loop's head start)."""
    v = [x for _, n, x in values if name_part in n][-last:]
    return (sum(v) / len(v), len(v)) if v else (None, 0)


def traffic_record(fetch_dir: str, write_dir: str, kernels: dict, last: int, calib_bytes: int,
                   calib_name: str = "copyBuffer") -> dict:
    """HBM bytes per launch of each kernel from FETCH_SIZE and WRITE_SIZE runs
    (KiB per dispatch), each scaled by the factor that makes the counter read
    calib_bytes for a plain copy of calib_bytes (the last copy kernel of the
    run).  kernels: {label: name_part}."""
    fv, wv = pmc_values(fetch_dir, "FETCH_SIZE"), pmc_values(write_dir, "WRITE_SIZE")
    fc = [x for _, n, x in fv if calib_name in n]
    wc = [x for _, n, x in wv if calib_name in n]
    if not fc or not wc:
        raise ValueError("no calibration copy in the counter runs")
    ff, wf = calib_bytes / (fc[-1] * 1024.0), calib_bytes / (wc[-1] * 1024.0)
    out = {"fetch_factor": round(ff, 4), "write_factor": round(wf, 4), "unit": "bytes per launch", "kernels": {}}
    for label, part in kernels.items():
        f, nf = loop_average(fv, part, last)
        w, nw = loop_average(wv, part, last)
        if f is None or w is None:
            continue
        out["kernels"][label] = {"fetch": round(f * 1024 * ff), "write": round(w * 1024 * wf),
                                 "total": round(f * 1024 * ff + w * 1024 * wf), "dispatches": min(nf, nw)}
    return out


def csrc_digest() -> str:
    """sha256 over the native sources (names and bytes), so a stored profile
    summary can tell whether it was taken on the current code."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def timeline_record(summaries: dict, command: str) -> dict:
    """Assemble per-mode timeline metrics ({mode: summary-json path}) into
    the stored record the benchmark reports."""
    modes = {}
    for mode, path in summaries.items():
        with open(path) as fh:
            t = json.load(fh)["timeline"]
        modes[mode] = {k: t.get(k) for k in ("mean_gap", "mean_kernel_gap", "mean_positive_kernel_gap", "gpu_idle_fraction",
                                             "compute_idle_fraction", "h2d_idle_fraction", "h2d_copies",
                                             "mean_stream_gap", "mean_intra_job_gap", "mean_job_boundary_gap",
                                             "span", "kernels", "mean_inter_batch_us")}
    return {"csrc_sha256": csrc_digest(), "command": command, "unit": "us", "modes": modes}


def summarize(dirpath: str, kernel: str = "", batch: int = 0, library_window: bool = False) -> dict:
    out = {"timeline": analyze_dir(dirpath, batch=batch, library_window=library_window),
           "kernel_stats": kernel_stats(dirpath)}
    if kernel:
        out["isolated"] = {kernel: isolated_run(dirpath, kernel)}
    return out


def traffic_file(out_path: str, runs: dict, calib_bytes: int = 64 << 20) -> dict:
    """Write the counter-traffic record the benchmark reads: runs maps a
    workload name to (fetch_dir, write_dir, probe_json) of a stage_probe
    --cold-only pair of counter runs; the average covers the cold loop's timed
    launches, the last `reps` dispatches of each kernel (reps from the probe's
    record)."""
    import hashlib
    kernels_src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "kernels.hip")
    rec = {"kernels_sha256": hashlib.sha256(open(kernels_src, "rb").read()).hexdigest(), "unit": "bytes per launch",
           "method": "rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE (KiB per dispatch), each scaled by the "
                     "factor that makes the counter read 64 MiB for the run's last plain 64 MiB device copy "
                     "(__amd_rocclr_copyBuffer); mean over the timed cold-loop dispatches of stage_probe "
                     "--cold-only (each kernel's last `reps` dispatches)",
           "workloads": {}}
    for name, (fdir, wdir, probe) in runs.items():
        line = [l for l in open(probe) if l.startswith("{")][-1]
        probe_rec = json.loads(line)
        slots = probe_rec["slots"]
        r = traffic_record(fdir, wdir, {"gauss5_f32": "k_gauss5", "sobel_thresh_f32": "k_sobel_thresh",
                                        "sobel_final": "k_sobel_final"}, last=int(probe_rec.get("reps", 100)),
                           calib_bytes=calib_bytes)
        r["slots"] = slots
        rec["workloads"][name] = r
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "traffic":
        # python -m ...trace traffic OUT.json NAME=FETCH_DIR,WRITE_DIR,PROBE_JSON ...
        runs = {a.split("=", 1)[0]: tuple(a.split("=", 1)[1].split(",")) for a in sys.argv[3:]}
        print(json.dumps(traffic_file(sys.argv[2], runs), indent=1))
    elif len(sys.argv) > 1 and sys.argv[1] == "timeline":
        # python -m ...trace timeline OUT.json "COMMAND" mode=summary.json ...
        rec = timeline_record(dict(a.split("=", 1) for a in sys.argv[4:]), sys.argv[3])
        with open(sys.argv[2], "w") as fh:
            json.dump(rec, fh, indent=1)
    elif len(sys.argv) > 1 and sys.argv[1] == "summarize":
        import argparse
        ap = argparse.ArgumentParser()
        ap.add_argument("cmd")
        ap.add_argument("dir")
        ap.add_argument("--kernel", default="")
        ap.add_argument("--batch", type=int, default=0)
        ap.add_argument("--library-window", action="store_true",
                        help="span from the first to the last library kernel only")
        a = ap.parse_args()
        print(json.dumps(summarize(a.dir, a.kernel, a.batch, a.library_window), indent=1))
    else:
        b = int(sys.argv[2]) if len(sys.argv) > 2 else 0
        print(json.dumps(analyze_dir(sys.argv[1], batch=b), indent=1))
