"""Host checks of bench.py: the one-GPU guard, and that the committed counter
summaries behind the roofline's `traffic` match the kernels' current sources."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import pytest  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_traffic_summaries_match_the_kernel_sources(monkeypatch):
    """Each dominant kernel has a committed counter summary with its HBM bytes and
    the SHA-256 of the sources it was taken from; a kernel edited since reports
    traffic = null (checked by changing the hash), and this test is then skipped
    with that reason until the counters are taken again."""
    stale = []
    for name, (_, srcs, fname) in bench.KERNELS.items():
        path = os.path.join(bench.PROFILES, fname)
        text = open(path).read()
        for key in ("sources_sha256", "fetch_bytes_per_launch", "write_bytes_per_launch"):
            assert key in text, f"{fname}: no {key}"
        t = bench.traffic_per_launch(name)
        if t is None:
            stale.append(name)
        else:
            assert t > 1e8, name  # at least the point records and the split partial sums
    monkeypatch.setattr(bench, "sources_sha256", lambda names: "0" * 64)
    for name in bench.KERNELS:
        assert bench.traffic_per_launch(name) is None
    if stale:
        pytest.skip("counter summaries taken from other sources (re-profile): " + ", ".join(stale))
