"""Host-side checks of bench.py: the one-GPU guard, the workload tables and
the rule that counter-based HBM traffic is reported only for the kernel
sources it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]


def test_every_workload_names_its_kernel_sources():
    for name, wl in bench.WORKLOADS.items():
        if name == "serve":  # many kernels per step; traffic is reported as null
            assert wl.key not in bench.KERNEL_SOURCES and bench.measured_traffic(wl.key) is None
            continue
        assert wl.key in bench.KERNEL_SOURCES, name
        for p in bench.KERNEL_SOURCES[wl.key]:
            assert os.path.exists(os.path.join(ROOT, p)), p


@pytest.mark.parametrize("key", sorted(bench.KERNEL_SOURCES))
def test_traffic_summary_is_tied_to_the_kernel_hash(key, monkeypatch):
    path = os.path.join(ROOT, "profiles", f"{key}_traffic.md")
    assert os.path.exists(path), f"no counter summary for {key}"
    text = open(path).read()
    assert "rocprofv3" in text and "FETCH_SIZE" in text and "WRITE_SIZE" in text
    h = bench.kernel_hash(key)
    assert len(h) == 16 and int(h, 16) >= 0
    t = bench.measured_traffic(key)
    if t is not None:  # counters taken on the current sources
        assert f"kernel_hash: `{h}`" in text or h in text
        assert t > 0
    # a summary whose hash differs from the sources is never reported
    monkeypatch.setattr(bench, "kernel_hash", lambda k="": "0" * 16)
    assert bench.measured_traffic(key) is None


@pytest.mark.parametrize("key", sorted(bench.KERNEL_SOURCES))
def test_kernel_stats_summary_gives_its_command(key):
    path = os.path.join(ROOT, "profiles", f"{key}_kernel_stats.md")
    assert os.path.exists(path), f"no kernel-trace summary for {key}"
    text = open(path).read()
    assert "rocprofv3" in text and "--kernel-trace" in text and "--stats" in text
    assert "_work/" not in text
