"""bench.py's host-side contract: more than one GPU is refused with a
message, and counter traffic is reported only for kernels the committed
summary covers, measured on the current kernel sources."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_lookup_follows_the_summary_and_the_sources(tmp_path, monkeypatch):
    assert bench.traffic_for("no_such_kernel") is None
    text = open(bench.TRAFFIC_PROFILE).read()
    names = [l.split("`")[1] for l in text.splitlines() if l.startswith("| `") and "_n11_" in l]
    assert names, "the committed summary lists the 2048-point kernels"
    if f"kernel sources sha256: {bench.kernel_sources_hash()}" in text:
        assert all(bench.traffic_for(n) > 0 for n in names)
    # the same summary with another source hash is not trusted
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace(bench.kernel_sources_hash(), "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(stale))
    assert all(bench.traffic_for(n) is None for n in names)
