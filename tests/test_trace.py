"""Timeline metrics against hand-computed timelines (tests/golden/trace_timelines.json)."""
import json
import os

import pytest

from paper_2606_05495_amd import trace

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "trace_timelines.json")))


@pytest.mark.parametrize("case", GOLD["cases"], ids=[c["name"] for c in GOLD["cases"]])
def test_timeline_metrics_golden(case):
    m = trace.timeline_metrics([tuple(x) for x in case["kernels"]], [tuple(x) for x in case["h2d"]],
                               [tuple(x) for x in case["d2h"]])
    for k in ("mean_kernel_gap", "mean_positive_kernel_gap", "span", "busy", "gpu_idle_fraction", "t_schedule",
              "compute_idle_fraction", "h2d_idle_fraction"):
        if k in case:
            assert m[k] == pytest.approx(case[k], abs=1e-12), k


def test_inter_batch_golden():
    ib = GOLD["inter_batch"]
    g = trace.inter_batch_gaps([tuple(x) for x in ib["h2d"]], [tuple(x) for x in ib["d2h"]], ib["batch"])
    assert g == pytest.approx(ib["gaps"])


def test_union_and_gap_invariants():
    import random
    rnd = random.Random(7)
    for _ in range(200):
        iv = []
        for _ in range(rnd.randint(1, 20)):
            a = rnd.uniform(0, 100)
            iv.append((a, a + rnd.uniform(0, 10)))
        u = trace.union_length(iv)
        span = max(b for _, b in iv) - min(a for a, _ in iv)
        assert 0 <= u <= span + 1e-9
        assert u <= sum(b - a for a, b in iv) + 1e-9
        # the gaps plus the busy union tile the kernel span exactly
        assert sum(trace.kernel_gaps(iv)) + u == pytest.approx(span)


def test_stream_gaps_hand_timeline():
    # two streams, each running one job: copy, stage, stage, copy, then the next job's copy
    ks = [(0, 10), (12, 20), (20, 25), (30, 40), (45, 55),      # stream A
          (0, 5), (5, 6), (9, 10), (10, 20), (20, 21)]           # stream B
    st = ["A"] * 5 + ["B"] * 5
    nm = ["copy", "gauss", "sobel", "copy", "copy", "copy", "gauss", "sobel", "copy", "copy"]
    g = trace.stream_gaps(ks, st, nm)
    assert g["streams"] == 2
    # A: 2, 0, 5, 5 ; B: 0, 3, 0, 0
    assert g["mean_stream_gap"] == pytest.approx(15 / 8)
    assert g["mean_job_boundary_gap"] == pytest.approx((5 + 0) / 2)
    assert g["mean_intra_job_gap"] == pytest.approx((2 + 0 + 5 + 0 + 3 + 0) / 6)
    # without names every pair counts as inside a job
    g2 = trace.stream_gaps(ks, st)
    assert g2["mean_job_boundary_gap"] is None and g2["mean_intra_job_gap"] == pytest.approx(15 / 8)


def test_stream_gaps_with_completion_word_kernel():
    # copy, stage, copy, flag | copy ... : the flag -> copy pair is the job boundary
    ks = [(0, 10), (11, 20), (22, 30), (30, 31), (40, 50), (50, 60)]
    nm = ["copy", "stage", "copy", "k_done_flag", "copy", "stage"]
    g = trace.stream_gaps(ks, ["A"] * 6, nm)
    assert g["mean_job_boundary_gap"] == pytest.approx(9.0)
    assert g["mean_intra_job_gap"] == pytest.approx((1 + 2 + 0 + 0) / 4)


def test_eq_terms_hand_timeline():
    # stream A: job 1 = copy(0,10) g(12,20) s(21,25) copy(27,30) flag(30,31); job 2 = copy(40,50) g(50,55) s(55,56) copy(60,62)
    # stream B: two chains interleaved on one stream (copy, copy, g, g, s, s, copy, copy) form a segment
    # with 4 stages, not the usual 2, and are skipped
    ks = [(0, 10), (12, 20), (21, 25), (27, 30), (30, 31), (40, 50), (50, 55), (55, 56), (60, 62),
          (0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 6), (6, 7), (7, 8)]
    st = ["A"] * 9 + ["B"] * 8
    nm = ["copy", "g", "s", "copy", "k_done_flag", "copy", "g", "s", "copy",
          "copy", "copy", "g", "g", "s", "s", "copy", "copy"]
    t = trace.eq_terms(ks, st, nm)
    assert t["jobs"] == 2
    assert t["t_in"] == pytest.approx((10 + 10) / 2)
    assert t["t_k"] == pytest.approx((8 + 4 + 5 + 1) / 2)
    assert t["t_out"] == pytest.approx((3 + 2) / 2)
    assert t["t_in_k"] == pytest.approx((2 + 0) / 2)
    assert t["delta_t_k"] == pytest.approx((1 + 0) / 2)
    assert t["t_k_out"] == pytest.approx((2 + 4) / 2)


def test_dma_copies_join_their_stream(tmp_path):
    """rocprofv3 CSVs where the input copies went by DMA (memory-copy trace,
    with its stream) and the rest as kernels: the per-job terms see
    [DMA input copy, stages, output copy kernel], the kernel gap only kernels,
    and the idle fraction the union of both."""
    k = tmp_path / "run_kernel_trace.csv"
    c = tmp_path / "run_memory_copy_trace.csv"
    # stream 7: job 1 = dma(0,10) g(12,20) s(21,25) k_copy(27,30); job 2 = dma(40,50) g(50,55) s(55,56) k_copy(60,62)
    krows = [(12, 20, "setrt::k_gauss"), (21, 25, "setrt::k_sobel"), (27, 30, "setrt::k_copy_out"),
             (50, 55, "setrt::k_gauss"), (55, 56, "setrt::k_sobel"), (60, 62, "setrt::k_copy_out")]
    with open(k, "w") as fh:
        fh.write('"Kind","Stream_Id","Kernel_Name","Start_Timestamp","End_Timestamp"\n')
        for a, b, n in krows:
            fh.write('"KERNEL_DISPATCH",7,"%s",%d,%d\n' % (n, a, b))
    with open(c, "w") as fh:
        fh.write('"Kind","Direction","Stream_Id","Start_Timestamp","End_Timestamp"\n')
        for a, b in ((0, 10), (40, 50)):
            fh.write('"MEMORY_COPY","MEMORY_COPY_HOST_TO_DEVICE",7,%d,%d\n' % (a, b))
    m = trace.analyze_dir(str(tmp_path))
    e = m["eq_terms"]  # ns in the files, us in the result
    assert e["jobs"] == 2
    assert e["t_in"] == pytest.approx(10 / 1e3)
    assert e["t_k"] == pytest.approx((8 + 4 + 5 + 1) / 2 / 1e3)
    assert e["t_in_k"] == pytest.approx((2 + 0) / 2 / 1e3)
    assert e["t_k_out"] == pytest.approx((2 + 4) / 2 / 1e3)
    # kernel gaps over the 6 kernels only: 1, 2, 20, 0, 4
    assert m["mean_kernel_gap"] == pytest.approx((1 + 2 + 20 + 0 + 4) / 5 / 1e3)
    # busy = [0,10] + [12,20] + [21,25] + [27,30] + [40,56] + [60,62] = 10+8+4+3+16+2 = 43 of 62
    assert m["gpu_idle_fraction"] == pytest.approx(1 - 43 / 62)
    # gaps with the DMA copies as GPU work: 2, 1, 2, 10, 0, 0, 4
    assert m["mean_gap"] == pytest.approx(19 / 7 / 1e3)
    assert m["h2d_copies"] == 2


def test_copy_kernels_give_copy_idle_and_batch_boundaries(tmp_path):
    """With copy kernels (k_copy_in / k_copy_out) and no DMA records, the
    input-copy idle fraction and Eq. 3's inter-batch gap come from the
    kernels: two batches of two jobs on one stream, the second starting 16
    after the first's last output copy."""
    k = tmp_path / "run_kernel_trace.csv"
    rows = [(0, 10, "k_copy_in"), (10, 20, "k_copy_in"), (20, 25, "k_g"), (25, 30, "k_g"),
            (30, 32, "k_copy_out"), (32, 34, "k_copy_out"),
            (50, 60, "k_copy_in"), (60, 70, "k_copy_in"), (70, 75, "k_g"), (75, 80, "k_g"),
            (80, 82, "k_copy_out"), (82, 84, "k_copy_out")]
    with open(k, "w") as fh:
        fh.write('"Kind","Stream_Id","Kernel_Name","Start_Timestamp","End_Timestamp"\n')
        for a, b, n in rows:
            fh.write('"KERNEL_DISPATCH",3,"setrt::%s",%d,%d\n' % (n, a, b))
    m = trace.analyze_dir(str(tmp_path), batch=2)
    assert m["mean_inter_batch_us"] == pytest.approx(16 / 1e3)
    # input copies busy 40 of the 84-long span
    assert m["h2d_idle_fraction"] == pytest.approx(1 - 40 / 84)
    assert m["h2d_copies"] == 0


def test_copy_overlap_fraction():
    """Input copies [0,10] and [20,30], output copies [5,25]: both directions
    busy for 5 + 5 = 10 of the 30 that either is."""
    assert trace.overlap_length([(0, 10), (20, 30)], [(5, 25)]) == pytest.approx(10)
    assert trace.overlap_length([(0, 10), (5, 12)], [(11, 20)]) == pytest.approx(1)
    assert trace.overlap_length([(0, 1)], [(2, 3)]) == 0
    assert trace.merged([(5, 6), (0, 2), (1, 3)]) == [(0, 3), (5, 6)]


def test_library_window_drops_setup_before_the_jobs(tmp_path):
    """A runtime copy kernel and a DMA copy long before the library's first
    kernel (a program's set-up uploads) count in the plain span; with the
    library window the span runs from the first to the last library kernel,
    and a copy overlapping the window's start is clipped to it."""
    k = tmp_path / "run_kernel_trace.csv"
    c = tmp_path / "run_memory_copy_trace.csv"
    krows = [(0, 5, "__amd_rocclr_copyBuffer"), (100, 110, "setrt::k_a"), (112, 120, "setrt::k_b"),
             (130, 140, "setrt::k_a")]
    with open(k, "w") as fh:
        fh.write('"Kind","Stream_Id","Kernel_Name","Start_Timestamp","End_Timestamp"\n')
        for a, b, n in krows:
            fh.write('"KERNEL_DISPATCH",1,"%s",%d,%d\n' % (n, a, b))
    with open(c, "w") as fh:
        fh.write('"Kind","Direction","Stream_Id","Start_Timestamp","End_Timestamp"\n')
        for a, b in ((10, 20), (95, 104)):
            fh.write('"MEMORY_COPY","MEMORY_COPY_HOST_TO_DEVICE",1,%d,%d\n' % (a, b))
    plain = trace.analyze_dir(str(tmp_path))
    # busy [0,5] [10,20] [95,110] [112,120] [130,140] = 5+10+15+8+10 = 48 of 140
    assert plain["gpu_idle_fraction"] == pytest.approx(1 - 48 / 140)
    win = trace.analyze_dir(str(tmp_path), library_window=True)
    # window [100,140]: busy [100,110] (copy clipped into it) [112,120] [130,140] = 28 of 40
    assert win["span"] == pytest.approx(40 / 1e3)
    assert win["gpu_idle_fraction"] == pytest.approx(1 - 28 / 40)
    assert win["h2d_copies"] == 1


def _pmc_csv(path, counter, rows):
    """A rocprofv3 --pmc counter file: rows of (dispatch id, kernel name, value);
    a dispatch may appear in several rows (one per XCD), which are summed."""
    import csv
    path.mkdir(parents=True, exist_ok=True)
    with open(path / "pmc_counter_collection.csv", "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, name, v in rows:
            wr.writerow([d, name, counter, v])


def test_traffic_record_scales_by_the_calibration_copy_and_averages_the_timed_loop(tmp_path):
    """Per-launch HBM bytes: counter KiB scaled so the last 64 MiB copy reads
    64 MiB, averaged over each kernel's last `last` dispatches (a cold loop's
    timed launches after the batch, the untimed pass and the head start).
    Values chosen so any other window or factor gives a different answer."""
    from paper_2606_05495_amd import trace
    mib64 = 64 << 20
    gauss = "void setrt::k_gauss5_win_f32<4, true>(setrt::GaussArgs)"
    fetch, write = [], []
    d = 0
    for i in range(10):  # earlier dispatches (batch, untimed pass): different values
        d += 1
        fetch.append((d, gauss, 999.0))
        write.append((d, gauss, 777.0))
    for i in range(4):  # the timed loop: each dispatch reported by two XCD rows
        d += 1
        fetch += [(d, gauss, 1000.0 + i), (d, gauss, 1000.0 + i)]
        write += [(d, gauss, 2048.0), (d, gauss, 2048.0)]
    d += 1
    fetch.append((d, "__amd_rocclr_copyBuffer", 32768.0))  # fetch counts half the copy's bytes
    write.append((d, "__amd_rocclr_copyBuffer", 65536.0))
    _pmc_csv(tmp_path / "f", "FETCH_SIZE", fetch)
    _pmc_csv(tmp_path / "w", "WRITE_SIZE", write)
    r = trace.traffic_record(str(tmp_path / "f"), str(tmp_path / "w"), {"gauss5_f32": "k_gauss5"}, last=4,
                             calib_bytes=mib64)
    assert r["fetch_factor"] == 2.0 and r["write_factor"] == 1.0
    k = r["kernels"]["gauss5_f32"]
    # fetch: mean of 2 x (1000..1003) KiB = 2003 KiB, times 2; write: 4096 KiB
    assert k["fetch"] == round(2003.0 * 1024 * 2.0)
    assert k["write"] == 4096 * 1024
    assert k["dispatches"] == 4
