"""The work per event quoted by the benchmark's roofline, recounted on the CPU.

tests/flopcount/count.cpp compiles the GPU library's own integrand headers for the
host with a counting binary64 scalar (add, sub, mul = 1, fma = 2, hardware estimate =
1, library functions at their FP64 FLOP prices measured on gfx950 by
tests/flopcount/ocml_price.hip under rocprofv3, bench.OCML_FLOP_PER_CALL; operations
on uniform values not counted) and runs it
over events drawn through a grid that the oracle adapted for five iterations.  The
result must equal the algorithmic FLOPs per event that bench.py uses for the event
kernel's roofline (to 0.5 %: the sampled events differ from the benchmark's)."""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
FC = os.path.join(HERE, "flopcount")


def _compiler():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++"), shutil.which("g++")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def counter(tmp_path_factory):
    cxx = _compiler()
    if cxx is None:
        pytest.skip("no C++ compiler")
    exe = str(tmp_path_factory.mktemp("fc") / "count")
    subprocess.run([cxx, "-std=c++20", "-O1", "-w", "-I", os.path.join(FC, "shim"),
                    "-I", os.path.join(ROOT, "paper_1503_06182_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                    "-o", exe, os.path.join(FC, "count.cpp")], check=True)
    return exe


def _prices():
    import bench
    return bench.OCML_FLOP_PER_CALL


KINDS = ("atan", "log", "exp", "expm1", "tan", "sincos", "sqrt", "div")


def prices(p, **over):
    """the counter's price arguments, in its order"""
    return [str(over.get(k, p[k])) for k in KINDS]


def count(exe, name, tmp_path, events=200_000):
    cfg = W.config(name)
    o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"])
    for _ in range(5):
        o.iterate(20_000)
        o.refine()
    grid = tmp_path / f"grid_{name}.txt"
    np.savetxt(grid, o.get_grid())
    p = _prices()
    r = subprocess.run([exe, name, str(grid), str(events)] + prices(p), check=True, capture_output=True, text=True)
    return json.loads(r.stdout)


@pytest.mark.parametrize("name", ["ww_4l", "w_plus", "ww_had"])
def test_algorithmic_flops_match_bench_constant(counter, name, tmp_path):
    import bench
    got = count(counter, name, tmp_path)
    want = bench.EVENT_KERNEL_WORK[(name, "fp64")]["algorithmic_f64"]
    assert abs(got["total"] / want - 1) < 5e-3, (name, got, want)
    assert got["nonzero"] > 0


def test_counting_scalar_counts_what_it_should(counter, tmp_path):
    """The count is the source's arithmetic with each mathematical function priced once:
    raising the price of one function moves the W+ total by exactly its calls per event
    times the change (one log per event; the W+W- integrand's tangents: two Breit-Wigner
    maps per event), the routines' own operations are not counted (with every price 0
    the W+W- total drops by more than its priced calls would explain otherwise), and
    uniform work is not counted."""
    p = _prices()
    cfg = W.config("w_plus")
    o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"])
    grid = tmp_path / "g.txt"
    np.savetxt(grid, o.get_grid())

    def run(proc, g, **over):
        return json.loads(subprocess.run([counter, proc, str(g), "20000"] + prices(p, **over), check=True,
                                         capture_output=True, text=True).stdout)

    base = run("w_plus", grid)
    one = run("w_plus", grid, log=p["log"] + 100)
    assert abs((one["total"] - base["total"]) - 100.0) < 1e-9      # exactly one log per event
    cw = W.config("ww_4l")
    ow = oracle.Vegas(cw["process"], cw["ndim"], cw["nbins"], cw["seed"], cw["alpha"], cw["params"])
    gw = tmp_path / "gw.txt"
    np.savetxt(gw, ow.get_grid())
    b = run("ww_4l", gw)
    t = run("ww_4l", gw, tan=p["tan"] + 10)
    assert abs((t["total"] - b["total"]) - 20.0) < 1e-9             # two tangents per event
    z = run("ww_4l", gw, **{k: 0 for k in KINDS})
    assert z["library_calls"] == 0.0 and z["total"] < b["total"] - b["library_calls"] + 1e-9
