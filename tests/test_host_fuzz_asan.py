"""AddressSanitizer run of the library's host code (skipped without hipcc, or with
NUMAG_ASAN=0).

Every source is rebuilt with -fsanitize=address on the host side only (device
code is compiled as usual and never runs: the fuzz driver calls
numag_workspace_size, which validates and plans without touching a GPU) and
20000 random or invalid requests are planned.  The sources compile in parallel
(about 10-60 s), so it runs in the default CPU suite: an invalid request that
crashes the planner (a division by zero, an access out of bounds) fails it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_18444_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.skipif(os.environ.get("NUMAG_ASAN") == "0" or not os.path.exists(HIPCC),
                                reason="needs hipcc (NUMAG_ASAN=0 switches it off)")


def test_workspace_size_planning_under_asan(tmp_path):
    from paper_2601_18444_amd.build import SOURCES
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC]
    procs, objs = [], []
    for src in SOURCES:
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err
    main = str(tmp_path / "fuzz_main.o")
    subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-I",
                    os.path.join(ROOT, "include"), "-x", "c++", "-c",
                    os.path.join(ROOT, "tests", "native", "fuzz_workspace_size.cpp"), "-o", main], check=True)
    exe = str(tmp_path / "fuzz")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", main, *objs, "-o", exe],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.startswith("ok ")
