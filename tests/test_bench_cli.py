"""Host-side checks of the benchmark script and the discharge-sweep helper
(no GPU needed): the one-GPU refusal, the profile summaries bench.py reads,
and argument validation."""
import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("name", sorted(os.path.basename(p) for p in __import__("glob").glob(
    os.path.join(ROOT, "profiles", "k_*_pmc.md"))))
def test_pmc_summaries_parse(name):
    """The machine-readable block bench.py takes roofline.traffic from."""
    txt = open(os.path.join(ROOT, "profiles", name)).read()
    d = json.loads(re.search(r"```json\s*(\{.*?\})\s*```", txt, re.S).group(1))
    for k in ("kernel", "steps_per_launch", "cells", "kernel_sha256_16", "hbm_bytes_per_launch",
              "algorithmic_bytes_per_launch", "fetch_scale", "write_scale"):
        assert k in d, k
    assert abs(d["hbm_bytes_per_launch"] - d["hbm_read_bytes_per_launch"]
               - d["hbm_write_bytes_per_launch"]) <= 2    # each rounded to whole bytes
    # one pass over the state per launch, whatever the steps per launch
    assert d["algorithmic_bytes_per_launch"] == 32 * d["cells"]
    # at least one pass over the state (20 B read, 12 B written per cell)
    assert d["hbm_read_bytes_per_launch"] >= 20 * d["cells"]
    assert d["hbm_write_bytes_per_launch"] >= 12 * d["cells"]


def test_sweep_rejects_bad_arguments():
    from paper_2204_10323_amd.sweep import discharge_sweep
    z = np.zeros((4, 4), np.float32)
    n = np.full((4, 4), 0.03, np.float32)
    with pytest.raises(ValueError):
        discharge_sweep(z, n, 1.0, (0, 0, 4, 1e-3), None, [1.0], 0, 0.1)
    with pytest.raises(ValueError):
        discharge_sweep(z, n, 1.0, (0, 0, 4, 1e-3), None, [1.0], 10, 0.0)
    with pytest.raises(ValueError):
        discharge_sweep(z, n, 1.0, (0, 0, 4, 1e-3), None, [1.0], 10, 0.1, mode="fastest")


def test_fraction_section():
    """Cells whose centre fraction (k + 1/2)/L lies in [f_start, f_end]."""
    from paper_2204_10323_amd import fraction_section
    assert fraction_section(10, 0.2, 0.5) == (2, 3)      # centres 0.25, 0.35, 0.45
    assert fraction_section(10, 0.0, 1.0) == (0, 10)
    assert fraction_section(10, 0.96, 1.0) == (0, 0)     # last centre is 0.95
    assert fraction_section(7, 0.5, 0.5) == (3, 1)       # the middle cell's centre is exactly 0.5
    assert fraction_section(4, 0.6, 0.4) == (0, 0)
    with pytest.raises(ValueError):
        fraction_section(0, 0.0, 1.0)
