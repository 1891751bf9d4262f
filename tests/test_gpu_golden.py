"""The 2048^2 valley (dx 5 m, meandering channel, triangular hydrograph peaking
at 500 m^3/s) after 20000 CFL steps as a HIP-graph-captured multi-step loop
with the clock on the device, FP32 on the GPU, against the FP64 oracle's
stored values (tests/golden/make_d2_golden.py): the depth of every cell, the
clock and the budget."""
import os
import sys

import numpy as np
import pytest

import paper_2204_10323_amd as fl
import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_d2_golden import input_hash  # noqa: E402


def test_valley2048_20000_steps_against_oracle_golden():
    g = np.load(os.path.join(HERE, "golden", "d2_2048_20000.npz"))
    sc = synth.config_d2()
    assert input_hash(sc) == str(g["input_sha256"]), "the input generator changed"
    print("CASE d2 20000 steps", flush=True)
    f = fl.from_scenario(sc, "f32")
    f.step(sc.steps)
    h = f.get_depth()
    r = f.get_report()
    f.close()
    ho = g["h_full"].astype(np.float64)
    assert ho.shape == h.shape == (sc.ny, sc.nx)
    assert (ho > 0.05).sum() > 100000, "the flood must cover a large part of the grid"
    err = np.abs(h.astype(np.float64) - ho)
    print(f"max|dh| over all {h.size} cells = {err.max():.3e} m", flush=True)
    assert err.max() <= 1e-3
    assert r.steps == int(g["steps"])
    assert abs(r.t / float(g["t"]) - 1) <= 1e-5
    assert abs(r.v_in / float(g["v_in"]) - 1) <= 1e-5
    assert abs(float(h.max()) - float(g["hmax"])) <= 1e-3
    assert r.budget_error() <= 1e-6
