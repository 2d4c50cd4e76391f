"""Host-side tests of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments before any GPU work (so these
run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "numag.h")
LIB = os.path.join(ROOT, "paper_2601_18444_amd", "libnumag.so")

if not os.path.exists(LIB):  # pragma: no cover
    pytest.skip("libnumag.so not built (run __graft_entry__.build())", allow_module_level=True)

from paper_2601_18444_amd import numag  # noqa: E402


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(numag_[a-z_0-9]+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert {"numag_amplitudes", "numag_cross_section", "numag_azimuthal_average", "numag_correlation",
            "numag_grad", "numag_workspace_size", "numag_last_error", "numag_version"} <= set(names)
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert "gfx950" in numag.version()


def _cpu_sample(W=10, K=1, offsets=None):
    s = numag.CSample()
    s.n_points = W
    s.pos = ctypes.c_void_p(0x1000) if W else None  # never dereferenced by validation
    s.nuc = None
    s.mag = None
    s.n_objects = K
    s.obj_offsets = offsets.ctypes.data_as(ctypes.c_void_p) if offsets is not None else None
    s.obj_pos = None
    s.regular = None
    return s


def _call_amp(sample, grid, rot=None, n_rot=1, mode=0, path=0, amp=0x2000, spec=None, ws=None, nws=0):
    r = rot.ctypes.data_as(ctypes.c_void_p) if rot is not None else None
    return numag._lib.numag_amplitudes(ctypes.byref(sample) if sample is not None else None, n_rot, r,
                                       ctypes.byref(grid) if grid is not None else None, path, mode, 0,
                                       ctypes.c_void_p(amp) if amp else None,
                                       ctypes.c_void_p(spec) if spec else None,
                                       ctypes.c_void_p(ws) if ws else None, nws, None)


def test_invalid_arguments_are_rejected_without_gpu_work():
    grid = numag.qgrid(0, 8, 8, 1.0)
    s = _cpu_sample()
    assert _call_amp(None, grid) == numag.E_INVALID
    assert "sample is NULL" in numag.last_error()
    assert _call_amp(s, None) == numag.E_INVALID
    assert _call_amp(s, numag.qgrid(0, 0, 8, 1.0)) == numag.E_INVALID
    assert _call_amp(s, numag.qgrid(0, 8, 8, -1.0)) == numag.E_INVALID
    assert _call_amp(s, numag.qgrid(7, 8, 8, 1.0)) == numag.E_INVALID
    bad = np.eye(3) * 1.01
    assert _call_amp(s, grid, rot=bad) == numag.E_INVALID
    assert "orthonormal" in numag.last_error()
    refl = np.diag([1.0, 1.0, -1.0])
    assert _call_amp(s, grid, rot=refl) == numag.E_INVALID
    assert _call_amp(s, grid, n_rot=2) == numag.E_INVALID
    assert _call_amp(s, grid, amp=None) == numag.E_INVALID  # amp_out required in COHERENT mode
    assert _call_amp(s, grid, mode=1, amp=None, spec=None) == numag.E_INVALID
    assert _call_amp(s, grid, mode=9) == numag.E_INVALID
    assert _call_amp(s, grid, path=1) == numag.E_INVALID  # separable needs a regular grid
    off = np.array([0, 4, 3, 10], dtype=np.int64)
    assert _call_amp(_cpu_sample(10, 3, off), grid) == numag.E_INVALID
    off = np.array([0, 4, 10], dtype=np.int64)
    assert _call_amp(_cpu_sample(11, 2, off), grid) == numag.E_INVALID


def test_workspace_size_and_too_small_workspace():
    grid = numag.qgrid(0, 64, 64, 1.0)
    s = _cpu_sample(W=100000)
    n = numag._lib.numag_workspace_size(ctypes.byref(s), 1, ctypes.byref(grid), 0, 0)
    assert n >= 100000 * 64
    assert _call_amp(s, grid, ws=0x3000, nws=1000) == numag.E_WORKSPACE
    assert "workspace too small" in numag.last_error()
    # degenerate sizes plan without dividing by zero (empty sample, 1x1 detector, polar)
    for W in (0, 1, 31, 33):
        for g in (numag.qgrid(0, 1, 1, 1.0), numag.qgrid(0, 3, 700, 1.0), numag.qgrid(1, 5, 9, 1.0)):
            e = _cpu_sample(W=W)
            n = numag._lib.numag_workspace_size(ctypes.byref(e), 1, ctypes.byref(g), 0, 0)
            assert n > 0, (W, g.kind)


def test_other_entry_points_validate():
    grid = numag.qgrid(0, 8, 8, 1.0)
    c = numag.consts()
    lib = numag._lib
    assert lib.numag_cross_section(ctypes.byref(grid), 1, None, None, ctypes.byref(c), 1, ctypes.c_void_p(8),
                                   None) == numag.E_INVALID
    assert lib.numag_cross_section(ctypes.byref(grid), 1, ctypes.c_void_p(8), None, ctypes.byref(c), 0,
                                   ctypes.c_void_p(8), None) == numag.E_INVALID
    bad = numag.consts(V=0.0)
    assert lib.numag_cross_section(ctypes.byref(grid), 1, ctypes.c_void_p(8), None, ctypes.byref(bad), 1,
                                   ctypes.c_void_p(8), None) == numag.E_INVALID
    assert lib.numag_azimuthal_average(ctypes.byref(grid), ctypes.c_void_p(8), 1, 0, 1.0, ctypes.c_void_p(8),
                                       None, None) == numag.E_INVALID
    pol = numag.qgrid(1, 8, 16, 1.0)
    assert lib.numag_azimuthal_average(ctypes.byref(pol), ctypes.c_void_p(8), 1, 7, 1.0, ctypes.c_void_p(8),
                                       None, None) == numag.E_INVALID
    assert lib.numag_correlation(None, None, 3, 1, None, 2, 1.0, None, None, None) == numag.E_INVALID
    # the half-detector path on a polar detector needs an even n_theta: the size query
    # refuses an odd one like the calls do (n_theta = 1 leaves no column to sum)
    pol1 = numag.qgrid(1, 8, 1, 1.0)
    s1 = _cpu_sample(W=10)
    for mode in (0, 1, 2):
        assert lib.numag_workspace_size(ctypes.byref(s1), 1, ctypes.byref(pol1), numag.PATH_DIRECT_HERMITIAN,
                                        mode) == 0
        assert "even n_theta" in numag.last_error()
    # no data sets: valid with NULL data and outputs, nothing launched
    assert lib.numag_cross_section(ctypes.byref(grid), 0, None, None, ctypes.byref(c), 1, None, None) == numag.OK
    assert lib.numag_cross_section(ctypes.byref(grid), 0, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.byref(c),
                                   1, None, None) == numag.E_INVALID
    assert lib.numag_cross_section(ctypes.byref(grid), 1, ctypes.c_void_p(8), None, ctypes.byref(c), 1, None,
                                   None) == numag.E_INVALID
    assert lib.numag_azimuthal_average(ctypes.byref(grid), None, 0, 4, 1.0, None, None, None) == numag.OK
    assert lib.numag_azimuthal_average(ctypes.byref(grid), None, 1, 4, 1.0, ctypes.c_void_p(8),
                                       None, None) == numag.E_INVALID
    assert lib.numag_azimuthal_average(ctypes.byref(grid), ctypes.c_void_p(8), 1, 4, 1.0, None,
                                       None, None) == numag.E_INVALID
    s = _cpu_sample()
    assert lib.numag_grad(ctypes.byref(s), None, ctypes.byref(grid), ctypes.byref(c), None, None, None, None,
                          None, None, None, 0, None) == numag.E_INVALID


def test_kernel_timer_without_launches():
    numag.kernel_timer(True)
    assert numag.kernel_timer_read(numag.KERNEL_DIRECT) == (0.0, 0)
    assert numag.kernel_timer_read(numag.KERNEL_OBJECTS) == (0.0, 0)
    numag.kernel_timer(False)
    assert numag._lib.numag_kernel_timer_read(3, None, None) == numag.E_INVALID
    assert numag._lib.numag_kernel_timer_read(-1, None, None) == numag.E_INVALID
    assert "unknown kernel" in numag.last_error()
    assert numag._lib.numag_kernel_timer_read(numag.KERNEL_ADJOINT, None, None) == numag.OK


def test_snapshots_validate_without_gpu_work():
    lib = numag._lib
    pts = numag.regular_grid((4, 5, 6), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    grid = numag.qgrid(0, 8, 8, 1.0)
    pol = numag.qgrid(1, 8, 8, 1.0)
    F64 = numag.PATH_SEPARABLE_F64
    assert lib.numag_snapshots_workspace_size(ctypes.byref(pts), 2, ctypes.byref(grid), F64) > 0
    assert lib.numag_snapshots_workspace_size(ctypes.byref(pts), 0, ctypes.byref(grid), F64) == 0
    assert lib.numag_snapshots_workspace_size(ctypes.byref(pts), 2, ctypes.byref(grid), numag.PATH_DIRECT) == 0
    assert lib.numag_snapshots_workspace_size(ctypes.byref(pts), 2, ctypes.byref(pol), F64) == 0
    assert lib.numag_snapshots_workspace_size(None, 2, ctypes.byref(grid), F64) == 0
    one = lib.numag_snapshots_workspace_size(ctypes.byref(pts), 1, ctypes.byref(grid), F64)
    two = lib.numag_snapshots_workspace_size(ctypes.byref(pts), 2, ctypes.byref(grid), F64)
    assert two > one
    # the Hermitian variant uses the FP64 path's workspace; path values end there
    H64 = numag.PATH_SEPARABLE_F64_HERMITIAN
    assert lib.numag_snapshots_workspace_size(ctypes.byref(pts), 2, ctypes.byref(grid), H64) == two
    assert lib.numag_snapshots_workspace_size(ctypes.byref(pts), 2, ctypes.byref(pol), H64) == 0
    assert lib.numag_snapshots_workspace_size(ctypes.byref(pts), 2, ctypes.byref(grid), H64 + 1) == 0
    bad = numag.regular_grid((0, 5, 6), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    assert lib.numag_snapshots_workspace_size(ctypes.byref(bad), 1, ctypes.byref(grid), F64) == 0
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.numag_amplitudes_snapshots(ctypes.byref(pts), 0, fake, None, ctypes.byref(grid), F64, fake, fake,
                                          1 << 20, None) == numag.E_INVALID
    assert lib.numag_amplitudes_snapshots(ctypes.byref(pts), 2, fake, None, ctypes.byref(grid), F64, None, fake,
                                          1 << 20, None) == numag.E_INVALID
    assert lib.numag_amplitudes_snapshots(ctypes.byref(pts), 2, fake, None, ctypes.byref(grid), F64, fake, fake,
                                          16, None) == numag.E_WORKSPACE
    assert "workspace too small" in numag.last_error()


def test_spectral_matrix_validates():
    lib = numag._lib
    grid = numag.qgrid(0, 8, 8, 1.0)
    assert lib.numag_spectral_matrix(ctypes.byref(grid), -1, None, None, None) == numag.E_INVALID
    assert lib.numag_spectral_matrix(ctypes.byref(grid), 2, None, ctypes.c_void_p(8), None) == numag.E_INVALID
    assert lib.numag_spectral_matrix(None, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == numag.E_INVALID
    assert lib.numag_spectral_matrix(ctypes.byref(grid), 0, None, None, None) == numag.OK


def test_hermitian_path_validates():
    s = _cpu_sample()
    pol_odd = numag.qgrid(1, 8, 9, 1.0)
    H = numag.PATH_DIRECT_HERMITIAN
    assert _call_amp(s, pol_odd, path=H, ws=0x3000, nws=1 << 30) == numag.E_INVALID
    assert "even n_theta" in numag.last_error()
    # object modes take the Hermitian path too, with the same even-n_theta rule
    assert _call_amp(s, pol_odd, path=H, mode=numag.MODE_DILUTE, amp=None, spec=0x4000, ws=0x3000,
                     nws=1 << 30) == numag.E_INVALID
    assert "even n_theta" in numag.last_error()
    grid = numag.qgrid(0, 8, 8, 1.0)
    assert _call_amp(s, grid, path=4, ws=0x3000, nws=1 << 30) == numag.E_INVALID
    assert numag._lib.numag_workspace_size(ctypes.byref(s), 1, ctypes.byref(grid), H, 0) > 0
    # the object workspace of the Hermitian path holds slots for half of the rows
    big = numag.qgrid(0, 64, 64, 1.0)
    full = numag._lib.numag_workspace_size(ctypes.byref(s), 3, ctypes.byref(big), numag.PATH_DIRECT, numag.MODE_DILUTE)
    half = numag._lib.numag_workspace_size(ctypes.byref(s), 3, ctypes.byref(big), H, numag.MODE_DILUTE)
    assert 0 < half < full


def test_binding_refuses_to_import_without_the_library(tmp_path):
    """No CPU fallback: a copy of the package without libnumag.so fails at import."""
    import shutil
    import subprocess
    import sys

    pkg = os.path.join(ROOT, "paper_2601_18444_amd")
    dst = tmp_path / "paper_2601_18444_amd"
    shutil.copytree(pkg, dst, ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__", "csrc"))
    code = "import paper_2601_18444_amd.numag"
    r = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "is not built" in r.stderr


def test_object_plans_validate_and_size_on_the_host():
    """numag_plan_create validates like numag_amplitudes (object modes only) and
    needs no device; numag_amplitudes_plan refuses a sample whose point count,
    object count or offsets differ from the plan's, and a short workspace, before
    any GPU work."""
    off = np.array([0, 4, 4, 10], dtype=np.int64)
    s = _cpu_sample(W=10, K=3, offsets=off)
    rots = np.stack([np.eye(3).reshape(9)] * 5)
    rp = rots.ctypes.data_as(ctypes.c_void_p)
    h = ctypes.c_void_p()
    for kind in (0, 1):
        grid = numag.qgrid(kind, 20, 24, 1.0)
        # coherent mode and the separable paths have no plan
        assert numag._lib.numag_plan_create(ctypes.byref(s), 5, rp, ctypes.byref(grid), 0, numag.MODE_COHERENT, 1,
                                            ctypes.byref(h)) == numag.E_INVALID
        assert numag._lib.numag_plan_create(ctypes.byref(s), 5, rp, ctypes.byref(grid), 1, numag.MODE_DILUTE, 1,
                                            ctypes.byref(h)) == numag.E_INVALID
        assert numag._lib.numag_plan_create(ctypes.byref(s), 5, rp, ctypes.byref(grid), 0, numag.MODE_SPLIT, 1,
                                            ctypes.byref(h)) == numag.E_INVALID  # SPLIT takes one rotation
        assert numag._lib.numag_plan_create(ctypes.byref(s), 5, rp, ctypes.byref(grid), 0, numag.MODE_DILUTE, 1,
                                            None) == numag.E_INVALID
        for path in (numag.PATH_DIRECT, numag.PATH_DIRECT_HERMITIAN):
            assert numag._lib.numag_plan_create(ctypes.byref(s), 5, rp, ctypes.byref(grid), path, numag.MODE_DILUTE,
                                                1, ctypes.byref(h)) == numag.OK, numag.last_error()
            nws = numag._lib.numag_plan_workspace_size(h)
            assert nws > 0 and nws % 256 == 0
            spec = ctypes.c_void_p(0x4000)
            ws = ctypes.c_void_p(0x8000)
            other = _cpu_sample(W=10, K=3, offsets=np.array([0, 5, 5, 10], dtype=np.int64))
            assert numag._lib.numag_amplitudes_plan(h, ctypes.byref(other), None, spec, ws, nws,
                                                    None) == numag.E_INVALID
            fewer = _cpu_sample(W=9, K=3, offsets=np.array([0, 4, 4, 9], dtype=np.int64))
            assert numag._lib.numag_amplitudes_plan(h, ctypes.byref(fewer), None, spec, ws, nws,
                                                    None) == numag.E_INVALID
            assert numag._lib.numag_amplitudes_plan(h, ctypes.byref(s), None, None, ws, nws, None) == numag.E_INVALID
            assert numag._lib.numag_amplitudes_plan(h, ctypes.byref(s), None, spec, ws, nws - 256,
                                                    None) == numag.E_WORKSPACE
            assert numag._lib.numag_plan_upload(h, ws, nws - 256, None) == numag.E_WORKSPACE
            numag._lib.numag_plan_destroy(h)
    numag._lib.numag_plan_destroy(None)
    assert numag._lib.numag_plan_workspace_size(None) == 0



def test_noalloc_entry_rejects_before_any_gpu_work():
    """numag_amplitudes_noalloc validates like numag_amplitudes and refuses detectors
    whose partial sums exceed half of its static scratch (no GPU needed: every case
    returns before a HIP call)."""
    lib = numag._lib
    s = _cpu_sample()
    amp = ctypes.c_void_p(0x2000)
    grid = numag.qgrid(0, 8, 8, 1.0)
    assert lib.numag_amplitudes_noalloc(ctypes.byref(s), 1, None, ctypes.byref(grid), numag.PATH_SEPARABLE_F64,
                                        amp, None) == numag.E_INVALID
    assert "path" in numag.last_error()
    assert lib.numag_amplitudes_noalloc(ctypes.byref(s), 1, None, ctypes.byref(grid), 0, None, None) == numag.E_INVALID
    assert lib.numag_amplitudes_noalloc(None, 1, None, ctypes.byref(grid), 0, amp, None) == numag.E_INVALID
    assert lib.numag_amplitudes_noalloc(ctypes.byref(s), 2, None, ctypes.byref(grid), 0, amp, None) == numag.E_INVALID
    bad = np.eye(3).reshape(9) * 2.0
    assert lib.numag_amplitudes_noalloc(ctypes.byref(s), 1, bad.ctypes.data_as(ctypes.c_void_p), ctypes.byref(grid),
                                        0, amp, None) == numag.E_INVALID
    odd = numag.qgrid(1, 8, 7, 1.0)
    assert lib.numag_amplitudes_noalloc(ctypes.byref(s), 1, None, ctypes.byref(odd), numag.PATH_DIRECT_HERMITIAN,
                                        amp, None) == numag.E_INVALID
    # partial sums of 64 bytes per evaluated pixel must fit in half of the scratch
    cap = 128 << 20
    limit = cap // 2 // 64
    big = numag.qgrid(0, 1025, 1024, 1.0)  # 1,049,600 > limit pixels
    assert 1025 * 1024 > limit
    assert lib.numag_amplitudes_noalloc(ctypes.byref(s), 1, None, ctypes.byref(big), 0, amp, None) == \
        numag.E_UNSUPPORTED
    assert "static scratch" in numag.last_error()
    text = open(HEADER).read()
    assert "#define NUMAG_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)" in text


def test_separable_hermitian_path_validates():
    """NUMAG_PATH_SEPARABLE_F64_HERMITIAN follows the separable paths' rules (a regular
    grid, one unrotated object, a Cartesian detector, coherent mode) and only the
    entry points that run separable paths accept it; path values end there.  Every
    case returns before any GPU work."""
    lib = numag._lib
    H64 = numag.PATH_SEPARABLE_F64_HERMITIAN
    grid = numag.qgrid(0, 8, 8, 1.0)
    pol = numag.qgrid(1, 8, 8, 1.0)
    s = _cpu_sample()
    assert _call_amp(s, grid, path=H64, ws=0x3000, nws=1 << 30) == numag.E_INVALID
    assert "regular" in numag.last_error()
    assert _call_amp(s, grid, path=H64 + 1, ws=0x3000, nws=1 << 30) == numag.E_INVALID
    assert "unknown path" in numag.last_error()
    reg = numag.regular_grid((4, 5, 6), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    sr = _cpu_sample(W=120)
    sr.pos = None
    sr.nuc = ctypes.c_void_p(0x1000)
    sr.regular = ctypes.cast(ctypes.pointer(reg), ctypes.c_void_p)
    assert lib.numag_workspace_size(ctypes.byref(sr), 1, ctypes.byref(grid), H64, 0) == \
        lib.numag_workspace_size(ctypes.byref(sr), 1, ctypes.byref(grid), numag.PATH_SEPARABLE_F64, 0) > 0
    assert _call_amp(sr, pol, path=H64, ws=0x3000, nws=1 << 30) == numag.E_INVALID
    assert "Cartesian" in numag.last_error()
    assert _call_amp(sr, grid, path=H64, mode=numag.MODE_DILUTE, amp=None, spec=0x4000, ws=0x3000,
                     nws=1 << 30) == numag.E_INVALID
    rot2 = np.stack([np.eye(3).reshape(9)] * 2)
    assert _call_amp(sr, grid, rot=rot2, n_rot=2, path=H64, ws=0x3000, nws=1 << 30) == numag.E_INVALID
    # the direct-only entry points refuse it
    c = numag.consts()
    fake = ctypes.c_void_p(0x5000)
    assert lib.numag_grad_path(ctypes.byref(s), None, ctypes.byref(grid), H64, ctypes.byref(c), None, fake, fake,
                               fake, fake, fake, fake, 1 << 30, None) == numag.E_INVALID
    assert "path" in numag.last_error()
    assert lib.numag_amplitudes_noalloc(ctypes.byref(s), 1, None, ctypes.byref(grid), H64,
                                        ctypes.c_void_p(0x2000), None) == numag.E_INVALID
    off = np.array([0, 4, 10], dtype=np.int64)
    so = _cpu_sample(W=10, K=2, offsets=off)
    h = ctypes.c_void_p()
    assert lib.numag_plan_create(ctypes.byref(so), 1, None, ctypes.byref(grid), H64, numag.MODE_DILUTE, 1,
                                 ctypes.byref(h)) == numag.E_INVALID
