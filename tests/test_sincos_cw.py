"""Accuracy of the FP64 sincos the sum kernels use in their generation phases
(Cody-Waite reduction by pi/2, Taylor polynomials on [-pi/4, pi/4]).

The same source is compiled for the host with hipcc and compared with the C
library's sin and cos (an independent implementation, correctly rounded to
within one ulp) on random arguments over the whole reduced range, on arguments
next to multiples of pi/2 (where the reduction cancels), at the quadrant
boundaries and up to the library fallback at 2^19.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_18444_amd", "csrc")
HIPCC = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if HIPCC is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("sincos") / "sincos_cw_check")
    src = os.path.join(ROOT, "tests", "native", "sincos_cw_check.cpp")
    res = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", CSRC, src, "-o", exe],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return exe


def _run(exe, xs):
    inp = "".join(float(x).hex() + "\n" for x in xs)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    s = np.array([float.fromhex(l.split()[0]) for l in out if l])
    c = np.array([float.fromhex(l.split()[1]) for l in out if l])
    return s, c


def _ulp_err(got, ref):
    # error in units of the last place of max(|ref|, 2^-30): absolute error for
    # values near zero, where sin x for x near k pi is itself tiny
    scale = np.maximum(np.abs(ref), 2.0 ** -30)
    return np.abs(got - ref) / (scale * 2.0 ** -52)


def test_random_arguments(checker):
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(-4, 4, 3000), rng.uniform(-200, 200, 3000),
                         rng.uniform(-5e5, 5e5, 2000), rng.uniform(-1e-3, 1e-3, 500)])
    s, c = _run(checker, xs)
    rs = np.array([math.sin(x) for x in xs])
    rc = np.array([math.cos(x) for x in xs])
    assert _ulp_err(s, rs).max() <= 4.0
    assert _ulp_err(c, rc).max() <= 4.0
    # unit modulus to a few ulp
    assert np.abs(s * s + c * c - 1.0).max() <= 8 * 2.0 ** -52


def test_near_multiples_of_half_pi_and_quadrant_edges(checker):
    ks = np.arange(-300, 301)
    base = ks * (math.pi / 2)
    xs = np.concatenate([base, np.nextafter(base, np.inf), np.nextafter(base, -np.inf),
                         base + math.pi / 4, base - math.pi / 4, [0.0, -0.0, 1e-300, -1e-300]])
    s, c = _run(checker, xs)
    rs = np.array([math.sin(x) for x in xs])
    rc = np.array([math.cos(x) for x in xs])
    # absolute error: at multiples of pi/2 one of the two is tiny
    assert np.abs(s - rs).max() <= 4 * 2.0 ** -52
    assert np.abs(c - rc).max() <= 4 * 2.0 ** -52
    # exact values at zero (signed)
    assert s[-4] == 0.0 and c[-4] == 1.0


def test_fallback_range_and_special_values(checker):
    xs = [2.0 ** 19 - 1.0, 2.0 ** 19, 2.0 ** 19 + 1.0, -(2.0 ** 19), 1e10, -3e15, math.inf, -math.inf, math.nan]
    s, c = _run(checker, xs)
    for x, a, b in zip(xs[:6], s[:6], c[:6]):
        assert abs(a - math.sin(x)) <= 4 * 2.0 ** -52 and abs(b - math.cos(x)) <= 4 * 2.0 ** -52, x
    assert np.isnan(s[6:]).all() and np.isnan(c[6:]).all()
