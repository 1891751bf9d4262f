"""The 2048^2 valley (dx 5 m, meandering channel, triangular hydrograph peaking
at 500 m^3/s) after 20000 CFL steps, FP32 on the GPU against the FP64 oracle's
stored values (tests/golden/make_d2_golden.py): sampled depths on a 16-cell
lattice and a dense 96 x 96 block at the channel, the clock and the budget."""
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
    stride, off = (int(v) for v in g["stride"])
    j0, i0 = (int(v) for v in g["block_origin"])
    hs = h[off::stride, off::stride].astype(np.float64)
    hb = h[j0:j0 + 96, i0:i0 + 96].astype(np.float64)
    assert (g["h_sample"] > 0.05).sum() > 200 and (g["h_block"] > 0.05).sum() > 100
    assert np.abs(hs - g["h_sample"]).max() <= 1e-3
    assert np.abs(hb - g["h_block"]).max() <= 1e-3
    assert r.steps == int(g["steps"])
    assert abs(r.t / float(g["t"]) - 1) <= 1e-5
    assert abs(r.v_in / float(g["v_in"]) - 1) <= 1e-5
    assert abs(float(h.max()) - float(g["hmax"])) <= 1e-3
    assert r.budget_error() <= 1e-6
