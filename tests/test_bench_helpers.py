"""CPU checks of the benchmark's own arithmetic: the roofline object, the
inverse-variance combination of the timed iterations, the history read back
from a checkpoint, and the refusal of a multi-GPU run (bench.py imports the
GPU stack only inside its workload functions)."""
import os
import struct
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_roofline_of_the_event_kernel():
    work = bench.EVENT_KERNEL_WORK[("w_plus", "fp64")]
    r = bench.roofline("w_plus", "fp64", 1_000_000, 33e-6)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    # the numerator is the algorithmic count; the executed count is reported beside it
    assert abs(r["achieved"] - work["algorithmic_f64"] * 1e6 / 33e-6 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 78.6) < 1e-12
    assert abs(r["valu_flop_utilisation"] - work["f64"] * 1e6 / 33e-6 / 1e12 / 78.6) < 1e-12
    assert r["traffic"] == work["traffic"]
    # the counters were taken at the workload's default size only
    assert bench.roofline("w_plus", "fp64", 500_000, 20e-6)["traffic"] is None
    # a mixed FP64 / FP32 kernel: the sum of each pipe's fraction of its own peak
    w = bench.EVENT_KERNEL_WORK[("ww_4l", "fp32me")]
    m = bench.roofline("ww_4l", "fp32me", 10_000_000, 5e-4)
    want = w["f64"] * 1e7 / 5e-4 / 1e12 / 78.6 + w["f32"] * 1e7 / 5e-4 / 1e12 / 157.3
    assert abs(m["frac"] - want) < 1e-12
    # no counted figure for this workload: nothing is claimed
    d = bench.roofline("dy_z", "fp64", 10_000, 9e-6)
    assert d["achieved"] is None and d["frac"] is None


def test_flow_layer_flop_count():
    """two products per event and layer: 128 x 128 and 128 x 188 (the 188 spline
    parameters; the kernel's padding to 192 columns is not work)"""
    assert bench.FLOW_LAYER_MFMA_FLOP == 2 * 128 * 128 + 2 * 128 * 188 == 80896


def test_combine_is_inverse_variance():
    I, s = bench.combine([(1.0, 0.04), (1.2, 0.01)])
    assert abs(I - (1.0 / 0.04 + 1.2 / 0.01) / (1 / 0.04 + 1 / 0.01)) < 1e-15
    assert abs(s - (1 / (1 / 0.04 + 1 / 0.01)) ** 0.5) < 1e-15


def test_history_from_checkpoint_layout():
    """header {magic, process, ndim, nbins, iter, seed, fold scales[4]}, edges, history"""
    ndim, nbins, hist = 2, 3, [(1.5, 0.25), (2.5, 0.5)]
    blob = struct.pack("<Q3iIQ4i", 0x5645474153434B32, 0, ndim, nbins, len(hist), 7, 1, 20, 40, 0)
    blob += struct.pack(f"<{ndim * (nbins + 1)}d", *([0.25] * (ndim * (nbins + 1))))
    blob += struct.pack(f"<{2 * len(hist)}d", *[v for p in hist for v in p])
    assert bench.history_from_state(blob, ndim, nbins) == hist


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
