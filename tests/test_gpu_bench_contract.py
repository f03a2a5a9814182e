"""bench.py's output line on the GPU: one JSON object with the metric, the
roofline of the dominant kernels and the CPU baseline, consistent with
itself (a short run of the headline workload)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_headline_line_keeps_the_contract():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
                        "--check", "2", "--cpu-sample", "16", "--single-sample", "8"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["unit"] == "pixels/s" and d["higher_is_better"] is True and d["dtype"] == "f32"
    assert d["value"] > 0 and abs(d["value"] * d["ms_per_step"] * 1e-3 - 4096) < 1e-6 * 4096
    assert "workload" in d["config"] and "model" not in d["config"]
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    assert rf["traffic"] is None or rf["traffic"] > 0
    assert 0.3 < rf["frac"] < 1.0
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["unit"] == "pixels/s"
    assert d["all_converged"] and d["l1_vs_oracle_max"] <= 1e-6
    assert d["l1_vs_oracle"]["pixels"] == 2 and d["l1_vs_oracle"]["of"] == 4096
    # the host-in-the-loop rate is reported beside value, never as it
    hi = d["host_inclusive"]
    assert hi["unit"] == "pixels/s" and 0 < hi["value"] < 1.2 * d["value"]  # timing noise of a 2-step run
    assert hi["pi_bytes_to_host"] == 4096 * 1024 * 4
