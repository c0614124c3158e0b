"""The kernels' own evaluations of atan, tan and sin/cos of 2 pi x, checked on the CPU.

tests/mathcheck/check.cpp compiles the GPU library's integrand headers for the host in
binary64 (the hardware reciprocal and inverse-square-root estimates, which the kernels
refine by Newton steps, taken as the exact operations) and compares atan_rr,
tan_halfpi and sincos_2pi with the C library's long double functions over the ranges
the integrands pass them.  The bars are the accuracy the per-event parity with the
oracle (1e-12 relative) was established with: about one unit in the last place for atan
and sin/cos, three for tan near the poles of its fold.
"""
import json
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def errors(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("clang++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    exe = str(tmp_path_factory.mktemp("mc") / "check")
    subprocess.run([cxx, "-std=c++17", "-O2", "-w", "-I", os.path.join(HERE, "mathcheck", "shim"),
                    "-I", os.path.join(ROOT, "paper_1503_06182_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                    "-o", exe, os.path.join(HERE, "mathcheck", "check.cpp")], check=True)
    out = subprocess.run([exe, "400000"], check=True, capture_output=True, text=True).stdout
    return json.loads(out)


def test_atan_within_one_ulp(errors):
    assert errors["atan"] <= 1.0, errors


def test_tan_within_three_ulp(errors):
    assert errors["tan"] <= 3.0, errors


def test_sincos_within_one_and_a_half_ulp(errors):
    assert errors["sin"] <= 1.5 and errors["cos"] <= 1.5, errors
