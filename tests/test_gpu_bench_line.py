"""bench.py end to end on a short run: the one JSON line carries every field
of its contract (metric, value, configuration, the roofline of the dominant
kernel with the PMC traffic of the current kernel sources, the CPU oracle
baseline), and its figures are consistent with each other."""
import json
import math
import os
import re
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    print("CASE bench.py --steps 4 (16384^2 pre-wetted start)", flush=True)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "4", "--warmup", "2",
           "--no-compare", "--no-ensemble", "--no-adjoint", "--no-sweep", "--no-active",
           "--no-variants", "--no-other-start", "--copy-gib", "1", "--cpu-budget", "1"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 4 and d["warmup"] == 2
    assert d["unit"] == "Gcell-updates/s" and d["higher_is_better"] is True
    assert d["dtype"] == "f32" and d["data"] == "synthetic" and d["vs_baseline"] is None
    assert d["config"]["workload"] == "valley_16384x16384_dx1m_prewetted"
    cells = d["config"]["cells"]
    assert cells == 16384 * 16384
    # value and ms_per_step describe the same time
    assert math.isclose(d["value"], cells / (d["ms_per_step"] / 1e3) / 1e9, rel_tol=2e-3)
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert math.isclose(rf["frac"], rf["achieved"] / rf["peak"], rel_tol=1e-3)
    spl = rf["steps_per_launch"]
    # one pass over the state per launch (read h z n qx qy, write h qx qy),
    # whatever the steps per launch; an HBM fraction cannot exceed 1
    assert rf["algorithmic_bytes_per_launch"] == 32 * cells
    assert rf["launches_timed"] == -(-d["steps"] // spl)
    assert math.isclose(rf["launch_ms"], d["ms_per_step"] * d["steps"] / rf["launches_timed"],
                        rel_tol=2e-3)
    assert math.isclose(rf["achieved"], rf["algorithmic_bytes_per_launch"] / (rf["launch_ms"] / 1e3) / 1e9,
                        rel_tol=2e-3)
    assert 0 < rf["frac"] < 1
    assert math.isclose(rf["one_pass_per_step_equivalent_gbs"], rf["achieved"] * spl, rel_tol=2e-3)
    # traffic comes from the committed PMC summary of the dominant kernel, and
    # only while that summary was taken on the current kernel sources
    sys.path.insert(0, ROOT)
    import bench
    summary = {}
    if os.path.exists(bench.PMC_SUMMARY[spl]):
        m = re.search(r"```json\s*(\{.*?\})\s*```", open(bench.PMC_SUMMARY[spl]).read(), re.S)
        summary = json.loads(m.group(1))
    fresh = summary.get("kernel_sha256_16") == d["extras"]["kernel_sha256_16"]
    fresh = fresh and summary.get("workload") == d["config"]["workload"]
    if fresh:
        assert rf["traffic"] == summary["hbm_bytes_per_launch"] and rf["traffic"] > 32 * cells
        assert 0 < rf["traffic_frac"] < 1
    else:
        assert rf["traffic"] is None
    cc = d["extras"]["copy_ceilings"]
    for k in ("kernel_copy_gbs", "hip_memcpy_d2d_gbs", "read_only_gbs", "write_only_gbs"):
        assert 0 < cc[k] < rf["peak"], k
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0
    assert cb["unit"] == d["unit"] and "oracle" in cb["sample"]
