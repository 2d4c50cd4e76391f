"""Pins of the oracle's Cartesian azimuthal binning (Sec. 2.5 eq. iqazi, read as
equal-width annuli of [0, q_max_avg]) and of its spectral-matrix packing
(Sec. 3.4 G_ab = A_a conj(A_b), packed as the C ABI states).

The binning pins read the oracle's complete pixel-to-annulus assignment: with
one indicator data set per pixel (f = e_p), the average of data set p is
1 / count(b) in the annulus b that holds pixel p and 0 in every other one.
That assignment is then checked against the annulus definition itself,
b dq <= |q| < (b + 1) dq, |q| = q_max_avg in the last annulus, |q| > q_max_avg
in none, on a detector whose axis values are small integers so that many |q|
fall exactly on annulus edges.  The mutation test builds copies of the
oracle with a plausible mistake planted in its binning (CPU only) and checks
that each of them fails these pins.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "numag_oracle.c")


def detector_axis(n, qmax):
    """Cartesian axis of the detector definition: q_i = -q_max + i (2 q_max / (n - 1))."""
    step = (2.0 * qmax) / (n - 1)
    return -qmax + np.arange(n, dtype=np.float64) * step


def pixel_moduli(n0, n1, qmax):
    ay, az = detector_axis(n0, qmax), detector_axis(n1, qmax)
    qy = np.repeat(ay, n1)
    qz = np.tile(az, n0)
    return np.sqrt(qy * qy + qz * qz)


def assignment(avg, n0, n1, qmax, n_bins, qmax_avg):
    """Annulus of every pixel (-1: none) and the counts, read from the averages of
    the P indicator data sets."""
    P = n0 * n1
    I, cnt = avg(n0, n1, qmax, np.eye(P), n_bins, qmax_avg)
    I = np.nan_to_num(I, nan=0.0)
    pos = I > 0
    assert np.all(pos.sum(axis=1) <= 1), "a pixel averaged into two annuli"
    b = np.where(pos.any(axis=1), np.argmax(pos, axis=1), -1)
    return b, cnt, I


def check_annuli(avg, n0, n1, qmax, n_bins, qmax_avg, exact):
    """Every pixel's annulus against the definition; exact=False allows the one
    rounding of |q| / dq at an annulus edge."""
    b, cnt, I = assignment(avg, n0, n1, qmax, n_bins, qmax_avg)
    qn = pixel_moduli(n0, n1, qmax)
    dq = qmax_avg / n_bins
    tol = 0.0 if exact else 4 * np.finfo(float).eps
    inside = qn <= qmax_avg * (1 + tol)
    outside = qn > qmax_avg * (1 + tol)
    assert np.all(b[outside] == -1), "a pixel beyond q_max_avg was averaged"
    if exact:
        assert np.all(b[qn <= qmax_avg] >= 0), "a pixel with |q| <= q_max_avg was dropped"
    sel = inside & (b >= 0)
    lo, hi = b[sel] * dq, (b[sel] + 1) * dq
    q = qn[sel]
    last = b[sel] == n_bins - 1
    assert np.all(q >= lo * (1 - tol)), "a pixel below its annulus"
    upper_ok = (q < hi * (1 + tol)) | (last & (q <= qmax_avg * (1 + tol)))
    assert np.all(upper_ok), "a pixel above its annulus"
    # counts are the pixels of each annulus; the indicator average is 1 / count
    assert np.array_equal(cnt, np.bincount(b[b >= 0], minlength=n_bins))
    for p in np.nonzero(b >= 0)[0]:
        assert I[p, b[p]] == 1.0 / cnt[b[p]]


def oracle_avg(orc):
    def avg(n0, n1, qmax, f, n_bins, qmax_avg):
        return orc.azimuthal_average(orc.CARTESIAN, n0, n1, qmax, f, n_bins, qmax_avg=qmax_avg)
    return avg


# the integer detector: n = 9 on [-4, 4] gives q in {-4, ..., 4}, so |q| is exact
# and on an annulus edge for every pixel on an axis and for (3, 4) -> 5
INTEGER_CASES = [(9, 9, 4.0, 4, 4.0), (9, 9, 4.0, 8, 4.0), (9, 9, 4.0, 5, 5.0), (9, 9, 4.0, 3, 3.0)]


@pytest.mark.parametrize("case", INTEGER_CASES)
def test_annuli_on_integer_detector_are_exact(orc, case):
    n0, n1, qmax, n_bins, qmax_avg = case
    check_annuli(oracle_avg(orc), n0, n1, qmax, n_bins, qmax_avg, exact=True)


def test_annuli_on_irregular_detectors(orc):
    for (n0, n1, qmax, n_bins, qmax_avg) in [(37, 50, 1.3, 23, 1.1), (16, 16, 2.0, 64, 2.0), (21, 7, 0.9, 5, 1.5)]:
        check_annuli(oracle_avg(orc), n0, n1, qmax, n_bins, qmax_avg, exact=False)


def test_annulus_means_of_radial_functions(orc):
    """f = |q| averages to a value inside its annulus [b dq, (b + 1) dq], and
    f = |q|^2 inside [b^2 dq^2, (b + 1)^2 dq^2]; the last annulus is closed at
    q_max_avg."""
    n0, n1, qmax, n_bins = 64, 64, 1.0, 40
    qn = pixel_moduli(n0, n1, qmax)
    I, cnt = orc.azimuthal_average(orc.CARTESIAN, n0, n1, qmax, np.stack([qn, qn * qn]), n_bins, qmax_avg=qmax)
    dq = qmax / n_bins
    ok = cnt > 0
    b = np.arange(n_bins)[ok]
    eps = 1e-14
    assert np.all(I[0, ok] >= b * dq - eps) and np.all(I[0, ok] <= (b + 1) * dq + eps)
    assert np.all(I[1, ok] >= (b * dq) ** 2 - eps) and np.all(I[1, ok] <= ((b + 1) * dq) ** 2 + eps)
    assert cnt.sum() == int(np.sum(qn <= qmax))


MUTANTS = {
    "round instead of floor": ("(int64_t)floor(qn / dq)", "(int64_t)round(qn / dq)"),
    "ceil instead of floor": ("(int64_t)floor(qn / dq)", "(int64_t)ceil(qn / dq)"),
    "annuli closed below": ("(int64_t)floor(qn / dq)", "(int64_t)(ceil(qn / dq) - 1.0 < 0 ? 0 : ceil(qn / dq) - 1.0)"),
    "q_max_avg excluded": ("if (qn > qmax_avg) { bin[p] = -1; continue; }",
                           "if (qn >= qmax_avg) { bin[p] = -1; continue; }"),
    "last edge dropped": ("if (b >= n_bins) b = n_bins - 1;", "if (b >= n_bins) { bin[p] = -1; continue; }"),
}


def build_mutant(tmp_path, name, old, new):
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, f"mutation site of '{name}' not found once"
    path = tmp_path / (name.replace(" ", "_") + ".c")
    path.write_text(src.replace(old, new))
    lib = tmp_path / (name.replace(" ", "_") + ".so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-o", str(lib),
                           str(path), "-lm"])
    return ctypes.CDLL(str(lib))


def mutant_avg(lib):
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    fn = lib.orc_azimuthal_average
    fn.argtypes = [ctypes.c_int, i64, i64, P, P, i64, P, i64, ctypes.c_double, P, P]
    fn.restype = None

    def avg(n0, n1, qmax, f, n_bins, qmax_avg):
        ay, az = detector_axis(n0, qmax), detector_axis(n1, qmax)
        qy = np.ascontiguousarray(np.repeat(ay, n1))
        qz = np.ascontiguousarray(np.tile(az, n0))
        f = np.ascontiguousarray(np.atleast_2d(f), dtype=np.float64)
        I = np.zeros((f.shape[0], n_bins))
        cnt = np.zeros(n_bins, dtype=np.int64)
        fn(0, n0, n1, qy.ctypes.data_as(P), qz.ctypes.data_as(P), f.shape[0], f.ctypes.data_as(P), n_bins,
           float(qmax_avg), I.ctypes.data_as(P), cnt.ctypes.data_as(P))
        return I, cnt
    return avg


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_binning_pins_reject_planted_mistakes(tmp_path, name):
    """Each planted mistake in the oracle's annulus assignment fails a pin above."""
    old, new = MUTANTS[name]
    avg = mutant_avg(build_mutant(tmp_path, name, old, new))
    failed = False
    for case in INTEGER_CASES:
        try:
            check_annuli(avg, *case, exact=True)
        except AssertionError:
            failed = True
            break
    assert failed, f"mutant '{name}' passes every binning pin"


def test_unmutated_copy_passes(tmp_path):
    """The mutation harness itself: an unmodified copy passes the pins."""
    src = open(ORACLE_SRC).read()
    path = tmp_path / "same.c"
    path.write_text(src)
    lib = tmp_path / "same.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-o", str(lib),
                           str(path), "-lm"])
    avg = mutant_avg(ctypes.CDLL(str(lib)))
    for case in INTEGER_CASES:
        check_annuli(avg, *case, exact=True)


def test_spectral_packing_all_sixteen_entries(orc):
    """G_ab = A_a conj(A_b) packed as [G00 G11 G22 G33, Re/Im of G01 G02 G03 G12
    G13 G23] (the packing the C ABI documents), summed over amplitude sets.  The
    expected entries are worked out by hand for A = (1, i, 2, 3 + i) and
    A' = (2i, 0, 1, -1)."""
    A = np.array([[[1, 1j, 2, 3 + 1j]], [[2j, 0, 1, -1]]], dtype=np.complex128)  # [sets][P = 1][4]
    one = orc.spectral(A[0])[0]
    assert np.array_equal(one, np.array([1, 1, 4, 10, 0, -1, 2, 0, 3, -1, 0, 2, 1, 3, 6, -2], dtype=float))
    both = orc.spectral(A)[0]
    assert np.array_equal(both, np.array([5, 1, 5, 11, 0, -1, 2, 2, 3, -3, 0, 2, 1, 3, 5, -2], dtype=float))
