"""Parity at the benchmark's full size and launch configuration (16384^2, dx 1 m).

Dry start, 1000 CFL steps (the benchmark's workload): for this many steps the
flood stays near the inflow section, every other cell stays exactly dry, and
the run is identical to the same run on a window around the inflow.  The
oracle runs that window; the test shows the window is large enough from each
side's own output (the oracle's outer band stays bitwise dry; the GPU grid
outside the window is exactly zero) and compares every cell.

Pre-wetted start (the benchmark's headline workload): every cell carries
water, so the oracle runs the whole 268 M-cell grid, for 24 steps; and 1000
steps against the oracle's stored values on a lattice of cells and dense
blocks (tests/golden/make_d3wet_golden.py).
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2204_10323_amd as fl
import synth
from gpu_util import max_abs, rel_err
from synth import WEST, Scenario

pytestmark = pytest.mark.gpu

N = 16384
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def d3_dry():
    print("CASE generating 16384^2 valley", flush=True)
    return synth.config_d3(N, wet=False)


@pytest.mark.parametrize("spl", [3, 2, 1])
def test_valley16384_dry_1000_steps_full_grid(d3_dry, spl):
    """spl = 3 is the benchmark's launch configuration (three steps per launch,
    default tiling); spl = 2 two steps per launch, 1 the single-step kernel."""
    sc = d3_dry
    print(f"CASE fullsize dry 1000 steps, {spl} step(s) per launch", flush=True)
    f = fl.from_scenario(sc, "f32", fusion=spl)
    f.step(1000)
    h = f.get_depth()
    qx, qy = f.get_discharge()
    r = f.get_report()
    f.close()
    assert r.steps == 1000 and r.budget_error() <= 1e-6

    side, first, count, slope, ts, qs = sc.inflow
    x1, y0, y1 = 400, first - 300, first + count + 300
    sub = Scenario("win", x1, y1 - y0, sc.dx, np.ascontiguousarray(sc.z[y0:y1, :x1]),
                   np.ascontiguousarray(sc.n[y0:y1, :x1]), np.zeros((y1 - y0, x1), np.float32),
                   (WEST, first - y0, count, slope, ts, qs), None, dt_max=sc.dt_max)
    o = oracle.Run(sub)
    o.step(1000)
    assert o.clock.steps == 1000
    band = 3
    assert not o.h[:band].any() and not o.h[-band:].any() and not o.h[:, -band:].any()
    # everything outside the window stays exactly dry and still on the GPU
    inside = np.zeros(h.shape, dtype=bool)
    inside[y0:y1, :x1] = True
    assert not h[~inside].any()
    qin = np.zeros(qx.shape, dtype=bool)
    qin[y0:y1, :x1 + 1] = True
    assert not qx[~qin].any()
    qyin = np.zeros(qy.shape, dtype=bool)
    qyin[y0:y1 + 1, :x1] = True
    assert not qy[~qyin].any()
    # every cell of the window
    assert o.h.max() > 0.5
    assert max_abs(h[y0:y1, :x1], o.h) <= 1e-3
    assert abs(r.t / o.clock.t - 1) <= 1e-5
    assert abs(r.v_in / o.clock.v_in - 1) <= 1e-5


def _prewetted(sc):
    z = sc.z
    eta0 = np.float32(np.percentile(z[::16, ::16], 30))
    h0 = np.maximum(eta0 - z, np.float32(0)).astype(np.float32)
    return Scenario("d3wet", sc.nx, sc.ny, sc.dx, z, sc.n, h0, sc.inflow, sc.outflow,
                    dt_max=sc.dt_max)


def test_valley16384_prewetted_24_steps_full_grid(d3_dry):
    """The benchmark's headline workload and launch configuration (three steps
    per launch, default tiling, speculated later dts): 8 launches, every cell
    and face against the oracle run on the whole grid; two steps per launch
    give the same bits."""
    wet = _prewetted(d3_dry)
    got = {}
    for spl in (3, 2):
        print(f"CASE fullsize prewetted 24 steps, {spl} steps per launch", flush=True)
        f = fl.from_scenario(wet, "f32", fusion=spl)
        f.step(24)
        h = f.get_depth()
        qx, qy = f.get_discharge()
        r = f.get_report()
        f.close()
        del f
        got[spl] = (h, qx, qy, r)
    for a, b in zip(got[3][:3], got[2][:3]):
        assert np.array_equal(a, b)
    assert got[3][3].t == got[2][3].t and got[3][3].v_in == got[2][3].v_in
    h, qx, qy, r = got[3]
    o = oracle.Run(wet)
    o.step(24)
    assert (o.h > 0).mean() > 0.2
    eh, eqx, eqy = max_abs(h, o.h), rel_err(qx, o.qx), rel_err(qy, o.qy)
    print(f"max|dh| = {eh:.3e} m, qx rel {eqx:.3e}, qy rel {eqy:.3e}", flush=True)
    assert eh <= 1e-4
    assert eqx <= 1e-4 and eqy <= 1e-4
    assert r.steps == 24 and abs(r.t / o.clock.t - 1) <= 1e-6
    assert abs(r.v_in / o.clock.v_in - 1) <= 1e-5
    assert r.budget_error() <= 1e-6


@pytest.mark.parametrize("spl", [3, 2])
def test_valley16384_prewetted_1000_steps_against_oracle_golden(d3_dry, spl):
    """The headline workload for its stated 1000 steps, in the benchmark's launch
    configuration (spl = 3; also 2), against the oracle's stored depths and face discharges
    (tests/golden/make_d3wet_golden.py) on a lattice of every 64th cell and four
    dense 256 x 256 blocks (inflow, mid-valley channel, outflow edge, shoreline)."""
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from make_d3wet_golden import input_hash
    g = np.load(os.path.join(HERE, "golden", "d3wet_16384_1000.npz"))
    wet = _prewetted(d3_dry)
    assert input_hash(wet) == str(g["input_sha256"]), "the input generator changed"
    print(f"CASE fullsize prewetted 1000 steps, {spl} steps per launch", flush=True)
    f = fl.from_scenario(wet, "f32", fusion=spl)
    f.step(1000)
    h = f.get_depth()
    qx, qy = f.get_discharge()
    r = f.get_report()
    f.close()
    st, off = (int(v) for v in g["lattice"])
    B = int(g["block_size"])
    qmax = float(g["qmax"])
    lat = (slice(off, None, st), slice(off, None, st))
    eh = max_abs(h[lat], g["h_lat"])
    eq = max(max_abs(qx[lat], g["qx_lat"]), max_abs(qy[lat], g["qy_lat"])) / qmax
    for b, (j, i) in enumerate(g["block_origin"]):
        eh = max(eh, max_abs(h[j:j + B, i:i + B], g["h_blocks"][b]))
        eq = max(eq, max_abs(qx[j:j + B, i:i + B + 1], g["qx_blocks"][b]) / qmax,
                 max_abs(qy[j:j + B + 1, i:i + B], g["qy_blocks"][b]) / qmax)
    print(f"max|dh| = {eh:.3e} m, max|dq|/max|q| = {eq:.3e}", flush=True)
    assert (g["h_lat"] > 0.05).sum() > 10000
    assert eh <= 1e-3
    assert eq <= 1e-3
    assert r.steps == int(g["steps"]) and abs(r.t / float(g["t"]) - 1) <= 1e-6
    assert abs(r.v_in / float(g["v_in"]) - 1) <= 1e-5
    assert abs(float(h.max()) - float(g["hmax"])) <= 1e-3
    assert r.budget_error() <= 1e-6


def test_valley16384_dry_1000_steps_active_tiles(d3_dry):
    """The benchmark workload with active-tile skipping: the same depths and
    discharges as computing every item, with a small fraction of the items
    computed at the end."""
    import torch
    sc = d3_dry
    print("CASE fullsize dry 1000 steps, active tiles", flush=True)
    res = []
    for active in (True, False):
        f = fl.from_scenario(sc, "f32", active_tiles=active, fusion=None if active else 2)
        f.step(1000)
        h = torch.empty((sc.ny, sc.nx), dtype=torch.float32, device="cuda")
        f.get_depth(h)
        qx, qy = f.get_discharge()
        r = f.get_report()
        items = f.active_items() if active else None
        f.close()
        res.append((h, qx, qy, r, items))
    a, b = res
    assert torch.equal(a[0], b[0])
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert (a[3].steps, a[3].t, a[3].v_in, a[3].v_out) == (b[3].steps, b[3].t, b[3].v_in, b[3].v_out)
    nxt, tot = a[4]
    assert 0 < nxt < 0.01 * tot


def test_valley16384_active_autotune_prefers_small_items_when_dry(d3_dry):
    """Under active tiles the autotuner times skipping steps: on the dry start
    (a few items near the inflow hold water) items of 2 cells per lane x 16 rows
    march faster than 4 x 32 (measured 55 against 83 us per step); the state is
    left as it is."""
    sc = d3_dry
    f = fl.from_scenario(sc, "f32", active_tiles=True)
    f.step(20)
    h0 = f.get_depth()
    best, ms = f.autotune([(4, 32), (2, 16)], 20)
    assert best == (2, 16), (best, ms)
    assert np.array_equal(f.get_depth(), h0)
    f.step(30)
    g = fl.from_scenario(sc, "f32", fusion=2)
    g.step(50)
    assert np.array_equal(f.get_depth(), g.get_depth())
    f.close()
    g.close()


def test_valley16384_dry_1000_steps_active_tiles_two_steps(d3_dry):
    """Active tiles with two steps per launch on the benchmark workload: the
    same state as computing every item."""
    import torch
    sc = d3_dry
    print("CASE fullsize dry 1000 steps, active tiles, two steps per launch", flush=True)
    hs = []
    for active in (True, False):
        f = fl.from_scenario(sc, "f32", active_tiles=active, fusion=2)
        f.step(1000)
        h = torch.empty((sc.ny, sc.nx), dtype=torch.float32, device="cuda")
        f.get_depth(h)
        r = f.get_report()
        f.close()
        hs.append((h, r))
    assert torch.equal(hs[0][0], hs[1][0])
    assert (hs[0][1].t, hs[0][1].v_in, hs[0][1].v_out) == (hs[1][1].t, hs[1][1].v_in, hs[1][1].v_out)


@pytest.mark.parametrize("cpt", [2, 1])
def test_valley16384_dry_active_tiles_list_mode(d3_dry, cpt):
    """Active tiles with the selected list (mode 2), 2 or 1 cells per lane x 8
    rows (272,384 or 561,152 work items: the latter scans the selection
    kernels' block counts first), on the benchmark workload: the same depths
    as computing every item."""
    import torch
    sc = d3_dry
    print(f"CASE fullsize dry 1000 steps, active tiles list mode cpt={cpt}", flush=True)
    hs = []
    for kw in (dict(active_tiles=2, cells_per_lane=cpt, rows_per_item=8), dict(fusion=2)):
        f = fl.from_scenario(sc, "f32", **kw)
        f.step(1000)
        h = torch.empty((sc.ny, sc.nx), dtype=torch.float32, device="cuda")
        f.get_depth(h)
        r = f.get_report()
        f.close()
        hs.append((h, r))
    assert torch.equal(hs[0][0], hs[1][0])
    assert (hs[0][1].t, hs[0][1].v_in) == (hs[1][1].t, hs[1][1].v_in)
