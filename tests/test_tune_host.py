"""Host-side tests of the launch-shape table (no GPU work): defaults, explicit
entries, validation, point-count classes and the NUMAG_AUTOTUNE_CACHE file."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2601_18444_amd", "libnumag.so")
if not os.path.exists(LIB):  # pragma: no cover
    pytest.skip("libnumag.so not built", allow_module_level=True)

from paper_2601_18444_amd import numag  # noqa: E402


@pytest.fixture(autouse=True)
def _clean_table():
    numag.tune_clear()
    yield
    numag.tune_clear()


def test_defaults_follow_the_detector():
    cart = numag.qgrid(0, 256, 256, 2.0)
    d, c, tuned = numag.tune_get(numag.TUNE_DIRECT, cart, 262144)
    assert d == c and not tuned
    assert d[0] == 32  # 8 x 32 columns cover 256
    assert numag.tune_get(numag.TUNE_DIRECT, numag.qgrid(0, 16, 60, 1.0), 10)[0][0] == 8
    # the half detector of the Hermitian path has its own key
    dh, _, _ = numag.tune_get(numag.TUNE_DIRECT, cart, 262144, path=numag.PATH_DIRECT_HERMITIAN)
    assert dh[0] == 32
    # polar: the 4-wave shape only for detectors of at most 32 q rows
    assert numag.tune_get(numag.TUNE_DIRECT, numag.qgrid(1, 20, 64, 1.0), 1000)[0][0] == 1
    assert numag.tune_get(numag.TUNE_DIRECT, numag.qgrid(1, 256, 256, 1.0), 1000)[0][0] in (0, 2, 3, 4)
    a = numag.tune_get(numag.TUNE_ADJOINT, cart, 262144)[0]
    assert a[0] == 0 and a[1] > 0


def test_set_get_and_point_classes():
    g = numag.qgrid(0, 256, 256, 2.0)
    numag.tune_set(numag.TUNE_DIRECT, g, 262144, (64, 3072))
    d, c, tuned = numag.tune_get(numag.TUNE_DIRECT, g, 262144)
    assert tuned and c == (64, 3072) and d[0] == 32
    # same half-octave class floor(2 log2 W): 2^18 .. 2^18.5
    assert numag.tune_get(numag.TUNE_DIRECT, g, 300000)[2]
    assert not numag.tune_get(numag.TUNE_DIRECT, g, 380000)[2]
    assert not numag.tune_get(numag.TUNE_DIRECT, g, 262144, path=numag.PATH_DIRECT_HERMITIAN)[2]
    assert not numag.tune_get(numag.TUNE_ADJOINT, g, 262144)[2]
    # target 0 means the default target
    numag.tune_set(numag.TUNE_DIRECT, g, 262144, (16, 0))
    d, c, _ = numag.tune_get(numag.TUNE_DIRECT, g, 262144)
    assert c == (16, d[1])
    numag.tune_set(numag.TUNE_DIRECT, g, 262144, None)
    assert not numag.tune_get(numag.TUNE_DIRECT, g, 262144)[2]


def test_invalid_shapes_are_rejected():
    cart = numag.qgrid(0, 64, 64, 1.0)
    pol = numag.qgrid(1, 256, 256, 1.0)
    for kernel, grid, shape in [(numag.TUNE_DIRECT, cart, (12, 0)), (numag.TUNE_DIRECT, cart, (128, 0)),
                                (numag.TUNE_DIRECT, pol, (5, 0)), (numag.TUNE_DIRECT, pol, (1, 0)),
                                (numag.TUNE_ADJOINT, cart, (8, 0)), (numag.TUNE_OBJECTS, pol, (32, 0)),
                                (numag.TUNE_DIRECT, cart, (32, -1))]:
        with pytest.raises(numag.NumagError):
            numag.tune_set(kernel, grid, 1000, shape)
    with pytest.raises(numag.NumagError):
        numag.tune_get(7, cart, 10)
    with pytest.raises(numag.NumagError):
        numag.tune_set(numag.TUNE_DIRECT, cart, -1, (8, 0))


def test_cache_file_is_read_on_first_lookup(tmp_path):
    path = tmp_path / "shapes.txt"
    # a 1000 x 1000 polar detector, W = 2.6e6 points: class floor(2 log2 W) = 42
    path.write_text("# comment\ngfx950 direct 1 1000 1000 42 4 1024 1.0 2.0\ngfx950 bogus 0 1 1 0 8 0 0 0\n")
    code = ("import sys; sys.path.insert(0, sys.argv[1]); from paper_2601_18444_amd import numag; "
            "g = numag.qgrid(1, 1000, 1000, 1.5); print(numag.tune_get(numag.TUNE_DIRECT, g, 2625870))")
    env = dict(os.environ, NUMAG_AUTOTUNE_CACHE=str(path))
    out = subprocess.run([sys.executable, "-c", code, ROOT], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().endswith("(4, 1024), True)")
