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
