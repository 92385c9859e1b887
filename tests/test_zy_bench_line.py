"""bench.py on the GPU: one short run of the default workload prints one JSON
line with every field of the benchmark record, a roofline object for the
dominant kernel and a same-GPU copy rate.  No timing thresholds: only the
record's shape and internal consistency are checked."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_default_bench_line(tmp_path):
    print("bench.py --steps 2 --warmup 1 --no-cpu-baseline", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
                        "--no-cpu-baseline"], capture_output=True, text=True, timeout=110, cwd=str(tmp_path))
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["unit"] == "Gpts/s" and d["value"] > 0 and d["higher_is_better"] is True
    assert d["dtype"] == "f32" and "workload" in d["config"]
    # value = 100 sweeps of 256^3 points per step / step time
    assert abs(d["value"] - 100 * 256 ** 3 / (d["ms_per_step"] * 1e-3) / 1e9) <= 0.01 * d["value"]
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["alg_bytes_per_launch"] == 48 * 256 ** 3
    assert abs(rf["achieved"] - rf["alg_bytes_per_launch"] / (rf["kernel_ms"] * 1e-3) / 1e9) <= 0.01 * rf["achieved"]
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert 0 < rf["frac"] < 1.0 and rf["launches_timed"] > 0
    # the per-launch time over the step's 100 launches fits inside the step
    assert rf["kernel_ms"] * 100 <= d["ms_per_step"] * 1.01
    assert rf["traffic"] is None or rf["traffic"] > 0
    assert rf["copy_gbs_same_gpu"] > 0
    assert abs(rf["frac_of_copy"] - rf["achieved"] / rf["copy_gbs_same_gpu"]) < 1e-3
    assert d["cpu_baseline"] is None  # skipped by the flag
