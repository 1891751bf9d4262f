"""The discharge sweep (flooded extent against inflow discharge, every discharge
a member of one batched launch) against the FP64 oracle run member by member:
depths to the FP32/FP64 gates, the flooded-cell classification wherever the
oracle's depth is clear of the threshold, and an extent that grows with the
discharge."""
import numpy as np
import pytest

import oracle
import paper_2204_10323_amd as fl
from paper_2204_10323_amd.sweep import discharge_sweep
from synth import EAST, WEST, Scenario, Valley, _f32, manning_field, valley_dem64, west_section

pytestmark = pytest.mark.gpu

Q = [5.0, 20.0, 50.0, 100.0, 200.0, 400.0]
DT, STEPS, THR = 0.5, 600, 0.1


def _valley():
    v = Valley(160, 96, 5.0, 5e-4, 2.0, 40.0, 0.3, seed=7, meander=True)
    z = _f32(valley_dem64(v))
    n = _f32(manning_field(v))
    first, count = west_section(v, 40.0)
    return v, z, n, (WEST, first, count, 5e-4), (EAST, 0, v.ny, 5e-4)


def _oracle_member(v, z, n, inflow, outflow, q):
    side, first, count, slope = inflow
    sc = Scenario(f"sweep_{q}", v.nx, v.ny, v.dx, z, n, np.zeros_like(z),
                  (side, first, count, slope, np.array([0.0]), np.array([q])), outflow,
                  dt_max=1.0, dt_fixed=DT)
    o = oracle.Run(sc)
    o.step(STEPS)
    return o


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_sweep_against_oracle(prec):
    v, z, n, inflow, outflow = _valley()
    print(f"CASE discharge sweep {prec}", flush=True)
    out = discharge_sweep(z, n, v.dx, inflow, outflow, Q, STEPS, DT, threshold=THR,
                          precision=prec, keep_depths=True)
    assert out["seconds"] == STEPS * DT and out["ms"] > 0 and out["mode"] in ("batch", "sequential")
    ext_o = []
    for k, q in enumerate(Q):
        o = _oracle_member(v, z, n, inflow, outflow, q)
        h = out["depth"][k].astype(np.float64)
        if prec == "f64":
            assert np.abs(h - o.h).max() <= 1e-10 * max(1.0, np.abs(o.h).max()), q
        else:
            assert np.abs(h - o.h).max() <= 1e-3, q
        clear = np.abs(o.h - THR) > 2e-3
        assert np.array_equal((h > THR)[clear], (o.h > THR)[clear]), q
        ext_o.append(int((o.h > THR).sum()))
        assert abs(out["v_in"][k] / (q * STEPS * DT) - 1) <= 1e-5, q
        assert out["budget_error"][k] <= (1e-12 if prec == "f64" else 1e-6), q
    # more water, more flooded ground
    assert all(a <= b for a, b in zip(ext_o, ext_o[1:])) and ext_o[-1] > ext_o[0]
    ext = list(out["flooded_cells"])
    assert all(a <= b for a, b in zip(ext, ext[1:]))
    assert out["flooded_area_m2"][-1] == ext[-1] * v.dx * v.dx


def test_sweep_members_equal_single_runs():
    """A sweep member is bit for bit the same run made alone."""
    v, z, n, inflow, outflow = _valley()
    out = discharge_sweep(z, n, v.dx, inflow, outflow, [30.0, 300.0], 200, DT, keep_depths=True,
                          tiling=(2, 16))
    side, first, count, slope = inflow
    for k, q in enumerate([30.0, 300.0]):
        f = fl.Flood(v.nx, v.ny, v.dx, "f32")
        f.set_dem(z)
        f.set_manning(n)
        f.set_inflow(side, first, count, slope, np.array([0.0]), np.array([q]))
        f.set_outflow(*outflow)
        f.set_params(dt_fixed=DT)
        f.commit()
        f.step(200)
        h = f.get_depth()
        f.close()
        assert np.array_equal(h, out["depth"][k])


@pytest.mark.parametrize("spe", [1, 2, 3])
def test_sweep_modes_agree(spe):
    """Batched (one, two or three steps per queue entry) and one-after-another
    members give the same bits."""
    v, z, n, inflow, outflow = _valley()
    qs = [15.0, 150.0, 600.0]
    b = discharge_sweep(z, n, v.dx, inflow, outflow, qs, 150, DT, keep_depths=True, mode="batch",
                        steps_per_entry=spe)
    assert b["steps_per_entry"] == spe
    s = discharge_sweep(z, n, v.dx, inflow, outflow, qs, 150, DT, keep_depths=True,
                        mode="sequential")
    assert b["mode"] == "batch" and s["mode"] == "sequential"
    for hb, hs in zip(b["depth"], s["depth"]):
        assert np.array_equal(hb, hs)
    assert np.array_equal(b["v_in"], s["v_in"])


def test_sweep_active_tiles_same_bits():
    """Members stepped with active-tile skipping give the bits of the batch."""
    v, z, n, inflow, outflow = _valley()
    qs = [15.0, 150.0, 600.0]
    b = discharge_sweep(z, n, v.dx, inflow, outflow, qs, 150, DT, keep_depths=True, mode="batch")
    a = discharge_sweep(z, n, v.dx, inflow, outflow, qs, 150, DT, keep_depths=True,
                        mode="sequential", active_tiles=True)
    for hb, ha in zip(b["depth"], a["depth"]):
        assert np.array_equal(hb, ha)
    # the outflow volume is summed over another work decomposition with
    # several steps per entry: FP64 rounding
    assert np.array_equal(b["v_in"], a["v_in"])
    assert np.allclose(b["v_out"], a["v_out"], rtol=1e-13, atol=0.0)


def test_sweep_batch_with_active_tiles_same_bits():
    v, z, n, inflow, outflow = _valley()
    qs = [15.0, 150.0, 600.0]
    s = discharge_sweep(z, n, v.dx, inflow, outflow, qs, 150, DT, keep_depths=True, mode="sequential")
    b = discharge_sweep(z, n, v.dx, inflow, outflow, qs, 150, DT, keep_depths=True, mode="batch",
                        active_tiles=True)
    assert b["mode"] == "batch"
    for hs, hb in zip(s["depth"], b["depth"]):
        assert np.array_equal(hs, hb)
    assert np.array_equal(s["v_in"], b["v_in"])
