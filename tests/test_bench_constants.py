"""The benchmark's work constants against the committed counter summary (CPU only).

bench.py prices the event kernel's roofline with per-event FLOPs and per-launch HBM
bytes measured by rocprofv3 counter runs; profiles/k_event_counters_flops_hbm.txt
holds the derived figures of those runs.  The two must agree, so that a kernel
change whose counters were retaken cannot leave the benchmark quoting the old ones.
"""
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUMMARY = os.path.join(ROOT, "profiles", "k_event_counters_flops_hbm.txt")

# derived-line prefix in the summary -> (workload, precision) key of bench.py
LINES = {"W+ (1e6 events):": ("w_plus", "fp64"),
         "W+W- partonic (1e7 events), FP64:": ("ww_4l", "fp64"),
         "W+W- hadronic, 10 dims (1e7 events), FP64:": ("ww_had", "fp64"),
         "W+W- partonic (1e7 events), FP32 matrix element:": ("ww_4l", "fp32me")}


def derived():
    text = open(SUMMARY).read()
    block = text[text.index("== derived"):]
    out = {}
    for line in block.splitlines():
        for prefix, key in LINES.items():
            if line.startswith(prefix):
                f64 = float(re.search(r"FP64 FLOP/event = ([\d.]+)", line).group(1))
                m32 = re.search(r"FP32 FLOP/event = ([\d.]+)", line)
                mb = re.search(r"= (\d+) B$", line)
                out[key] = (f64, float(m32.group(1)) if m32 else 0.0, int(mb.group(1)) if mb else None)
    return out, block


def test_event_kernel_work_matches_counter_summary():
    got, _ = derived()
    assert set(got) == set(bench.EVENT_KERNEL_WORK), (sorted(got), sorted(bench.EVENT_KERNEL_WORK))
    for key, (f64, f32, byt) in got.items():
        w = bench.EVENT_KERNEL_WORK[key]
        assert abs(w["f64"] - f64) < 0.05 and abs(w["f32"] - f32) < 0.05, (key, w, f64, f32)
        assert w["traffic"] == byt, (key, w["traffic"], byt)


def test_histogram_stage_traffic_matches_counter_summary():
    _, block = derived()
    for prefix, key in (("W+ histogram stage", ("w_plus", 1_000_000)),
                        ("W+W- histogram stage", ("ww_4l", 10_000_000))):
        line = [x for x in block.splitlines() if x.startswith(prefix)][0]
        byt = int(re.search(r"= (\d+) B$", line).group(1))
        assert bench.HIST_STAGE_TRAFFIC[key] == byt, (key, byt)


def test_adjoint_work_matches_its_summary():
    text = open(os.path.join(ROOT, "profiles", "k_dy_grad_adjoint_64x1e6_trace_counters.txt")).read()
    f64 = float(re.search(r"FP64 FLOP per \(event, point\) = ([\d.]+)", text).group(1))
    assert abs(bench.ADJOINT_KERNEL_WORK["f64"] - f64) < 0.05
