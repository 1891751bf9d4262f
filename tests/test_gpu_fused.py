"""Two and three steps per launch (fl_set_fusion) against one step per launch.

Both make every step with the same dt, inflow and arithmetic, so the state,
clock and inflow volume must agree bit for bit, whatever the speculated dts
of the later steps turned out to be (kept, redone from the first wrong one,
or shorter launches while the CFL bound is close to active).  The outflow
volume is summed over a different work decomposition, so it agrees to FP64
rounding."""
import numpy as np
import pytest

import paper_2204_10323_amd as fl
import synth
from synth import EAST, NORTH, SOUTH, WEST, Scenario, config_d1, random_tiny

pytestmark = pytest.mark.gpu


def _run(sc, prec, fusion, chunks, advance=None, **params):
    f = fl.from_scenario(sc, prec, fusion=fusion, **params)
    for n in chunks:
        if isinstance(n, float):
            f.advance(n)
        else:
            f.step(n)
    h = f.get_depth()
    qx, qy = f.get_discharge()
    r = f.get_report(check=False)
    f.close()
    return h, qx, qy, r


def _same(a, b, what=""):
    for x, y, nm in zip(a[:3], b[:3], ("h", "qx", "qy")):
        assert np.array_equal(x, y, equal_nan=True), f"{what}: {nm} differs"
    ra, rb = a[3], b[3]
    assert ra.steps == rb.steps and ra.t == rb.t and ra.last_dt == rb.last_dt, what
    assert ra.done == rb.done and ra.nonfinite == rb.nonfinite, what
    assert ra.v_in == rb.v_in, what
    assert abs(ra.v_out - rb.v_out) <= 1e-13 * max(1.0, abs(rb.v_out)), what


@pytest.mark.parametrize("k,prec,cpt", [(2, "f32", 1), (2, "f32", 2), (2, "f32", 4), (2, "f64", 1),
                                        (2, "f64", 2), (3, "f32", 1), (3, "f32", 2), (3, "f64", 1),
                                        (3, "f64", 2)])
def test_valley256_2000_steps(k, prec, cpt):
    sc = config_d1()
    print(f"CASE valley256 k={k} {prec} cpt={cpt}", flush=True)
    ref = _run(sc, prec, 1, [2000])
    got = _run(sc, prec, (k, cpt, 0), [2000])
    _same(got, ref, f"k={k} {prec} cpt={cpt}")
    assert got[3].v_out > 0 and got[3].steps == 2000


@pytest.mark.parametrize("seed", range(12))
def test_tiny_grids_every_side(seed):
    """Ragged tiny grids, random wet/dry state and boundary sections, several
    calls of lengths not multiples of 2 or 3, FP32 and FP64, two and three
    steps per launch."""
    rng = np.random.default_rng(seed)
    nx, ny = int(rng.integers(1, 140)), int(rng.integers(1, 90))
    sc = random_tiny(nx, ny, 100 + seed)
    chunks = [7, 1, 10, 2, 5]
    for prec in ("f32", "f64"):
        ref = _run(sc, prec, 1, chunks)
        for k, rows in ((2, 8), (3, 5)):
            print(f"CASE tiny {nx}x{ny} seed {seed} {prec} k={k}", flush=True)
            got = _run(sc, prec, (k, 1 + seed % 2, rows), chunks)
            _same(got, ref, f"tiny {nx}x{ny} {prec} k={k}")


def _filling_basin(nx=96, ny=64, dt_max=1.0, q=400.0):
    """A small basin at 1 m filled from the west: with dt_max = 1 s the CFL
    bound becomes active once the deepest cell passes 5 cm, during the first
    launches -- the speculated second dt is wrong, steps are redone, then
    launches make one step while the bound stays active."""
    z = synth._f32(np.fromfunction(lambda j, i: 0.002 * (nx - i) + 0.01 * np.sin(j / 5.0),
                                   (ny, nx)))
    n = np.full((ny, nx), 0.03, np.float32)
    ts = np.array([0.0, 50.0, 100.0])
    qs = np.array([q, q, 0.0])
    return Scenario("basin", nx, ny, 1.0, z, n, np.zeros_like(z),
                    (WEST, 20, 8, 1e-3, ts, qs), (EAST, 0, ny, 1e-3), dt_max=dt_max)


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_cfl_becomes_active(prec, k):
    sc = _filling_basin()
    print(f"CASE basin {prec} k={k}", flush=True)
    ref = _run(sc, prec, 1, [150, 151])
    got = _run(sc, prec, (k, 1, 8), [150, 151])
    _same(got, ref, prec)
    assert ref[3].last_dt < sc.dt_max     # the bound is active at the end


@pytest.mark.parametrize("k", [2, 3])
def test_cfl_activates_at_each_step_of_a_launch(k):
    """The bound becomes active after the first, second or third step of a
    launch, in basins filled at different rates: every kind of redo."""
    for q in (150.0, 260.0, 410.0, 700.0):
        sc = _filling_basin(q=q)
        print(f"CASE basin q={q} k={k}", flush=True)
        chunks = [37, 50, 64]
        ref = _run(sc, "f32", 1, chunks)
        got = _run(sc, "f32", (k, 2, 6), chunks)
        _same(got, ref, f"q={q} k={k}")


@pytest.mark.parametrize("k", [2, 3])
def test_t_end_inside_a_launch(k):
    sc = config_d1()
    for t_end in (123.4, 123.9, 124.6):
        ref = _run(sc, "f32", 1, [301], t_end=t_end)
        got = _run(sc, "f32", (k, 2, 0), [301], t_end=t_end)
        _same(got, ref)
        assert got[3].done == 1 and got[3].t == t_end


@pytest.mark.parametrize("k", [2, 3])
def test_fixed_dt_valley(k):
    sc = synth.config_d5(nx=256, steps=400)
    ref = _run(sc, "f32", 1, [400])
    got = _run(sc, "f32", (k, 2, 0), [400])
    _same(got, ref)


@pytest.mark.parametrize("k", [2, 3])
def test_nonfinite_stops_the_clock(k):
    nx, ny = 40, 12
    z = np.zeros((ny, nx), np.float32)
    n = np.full((ny, nx), 0.03, np.float32)
    sc = Scenario("blowup", nx, ny, 1.0, z, n, np.zeros_like(z),
                  (WEST, 0, ny, 1e-3, np.array([0.0]), np.array([1e38])), None, dt_max=0.1)
    for fixed in (0.0, 0.1):
        sc.dt_fixed = fixed
        ref = _run(sc, "f32", 1, [12])
        got = _run(sc, "f32", (k, 1, 0), [12])
        _same(got, ref)
        assert got[3].nonfinite == 1


@pytest.mark.parametrize("k", [2, 3])
def test_mixed_with_single_steps_and_advance(k):
    """fl_step(1) (single-step launch), fl_advance (single-step launches) and
    multi-step runs in any order continue the same state."""
    sc = config_d1()
    seq = [1, 9, 5.0, 40, 1, 1, 33, 2, 4]
    ref = _run(sc, "f32", 1, seq)
    got = _run(sc, "f32", (k, 2, 0), seq)
    _same(got, ref)


@pytest.mark.parametrize("k", [2, 3])
def test_batch_after_multi_step_run(k):
    """A context stepped by multi-step launches can join a batch: the buffer
    parity handed back to the single-step path is consistent."""
    sc = config_d1()
    ref = _run(sc, "f32", 1, [31])
    f = fl.from_scenario(sc, "f32", fusion=(k, 2, 0))
    f.step(11)
    b = fl.Batch([f])
    b.run(20)
    b.close()
    h = f.get_depth()
    qx, qy = f.get_discharge()
    r = f.get_report()
    f.close()
    _same((h, qx, qy, r), ref)


def test_valley4096_benchmark_construction():
    """The benchmark's 1 m construction at 4096^2, 60 steps, two steps per
    launch at CPT 2 and 4, three at CPT 2 (the default 48 rows and 16)."""
    sc = synth.config_d3(4096)
    ref = _run(sc, "f32", 1, [60])
    for k, cpt, rows in ((2, 2, 0), (2, 4, 0), (3, 2, 0), (3, 2, 16)):
        print(f"CASE valley4096 k={k} cpt={cpt} rows={rows}", flush=True)
        got = _run(sc, "f32", (k, cpt, rows), [60])
        _same(got, ref, f"k={k} cpt={cpt}")


@pytest.mark.parametrize("k", [2, 3])
def test_autotune_fusion_keeps_the_bits(k):
    """Frozen trial steps of both launch modes leave the state as it is; the
    run continues bit for bit with whichever mode was kept."""
    sc = config_d1()
    ref = _run(sc, "f32", 1, [400])
    f = fl.from_scenario(sc, "f32", fusion=(k, 2, 0))
    f.step(100)
    spl, ms = f.autotune_fusion(20)
    assert spl in (1, k) and ms > 0
    f.step(300)
    h = f.get_depth()
    qx, qy = f.get_discharge()
    r = f.get_report(check=False)
    f.close()
    _same((h, qx, qy, r), ref)
    g = fl.from_scenario(sc, "f32")              # committed without the two-step buffers
    assert fl.lib().fl_autotune_fusion(g.ctx, 10, None, None) == fl.FL_ESTATE
    g.close()


def test_autotune_fusion_picks_multi_step_on_the_benchmark_grid():
    """On the 16384^2 benchmark grid (dry start) several steps per launch win."""
    sc = synth.config_d3(16384)
    for k in (2, 3):
        f = fl.from_scenario(sc, "f32", fusion=k)
        spl, ms = f.autotune_fusion(20)
        f.close()
        assert spl == k, ms


def test_three_steps_refusals():
    """Three steps per launch: not at 4 cells per lane, and with active tiles
    not with items of fewer than three rows; steps per launch above 3 are
    refused."""
    sc = config_d1()
    f = fl.Flood(sc.nx, sc.ny, sc.dx, "f32")
    with pytest.raises(fl.FloodError):
        f.set_fusion(4)
    f.close()
    for kw in (dict(fusion=(3, 4, 0)), dict(fusion=(3, 2, 2), active_tiles=True)):
        with pytest.raises(fl.FloodError):
            fl.from_scenario(sc, "f32", **kw).close()
    fl.from_scenario(sc, "f32", fusion=3, active_tiles=True).close()
