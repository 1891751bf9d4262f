"""GPU parity: libflood (HIP, gfx950) against the FP64 CPU oracle, through the C interface.

Gates (from the accuracy targets of the method's build):
  * FP64 GPU build vs oracle: max|dh| / max|h| and max|dq| / max|q| <= 1e-10;
  * FP32 GPU build vs oracle: max|dh| <= 1e-3 m after the stated step counts;
  * FP64 volume budget of the FP32 build closes to <= 1e-6 relative;
  * different launch tilings give bit-identical results (a face computed by
    two work items gets the same bits).
Both sides start from the same float32-rounded inputs of the seeded generator.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2204_10323_amd as fl
from gpu_util import max_abs, rel_err, run_gpu, run_oracle
from synth import (EAST, NORTH, SOUTH, WEST, Scenario, config_d1, random_tiny)

pytestmark = pytest.mark.gpu


def _print_case(*a):
    print("CASE", *a, flush=True)


# ------------------------------------------------------------- tiny brute force
TINY = [(1, 1), (2, 1), (1, 3), (3, 2), (5, 4), (7, 9), (9, 7), (4, 8)]


@pytest.mark.parametrize("nx,ny", TINY)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_step_by_step_fp64(nx, ny, seed):
    """Random wet/dry tiny grids with random boundary sections, every step compared (FP64)."""
    sc = random_tiny(nx, ny, seed * 100 + nx * 10 + ny)
    _print_case("tiny64", nx, ny, seed)
    f = fl.from_scenario(sc, "f64", steps_per_graph=6)
    o = oracle.Run(sc)
    for step in range(12):
        f.step(1)
        o.step(1)
        h = f.get_depth()
        qx, qy = f.get_discharge()
        sh = max(np.abs(o.h).max(), 1e-3)
        sq = max(np.abs(o.qx).max(), np.abs(o.qy).max(), 1e-3)
        assert max_abs(h, o.h) <= 1e-12 * sh, (step, max_abs(h, o.h))
        assert max_abs(qx, o.qx) <= 1e-12 * sq, step
        assert max_abs(qy, o.qy) <= 1e-12 * sq, step
    r = f.get_report()
    assert abs(r.t - o.clock.t) <= 1e-12 * max(1.0, o.clock.t)
    assert r.steps == o.clock.steps
    f.close()


@pytest.mark.parametrize("nx,ny", TINY)
def test_tiny_step_by_step_fp32(nx, ny):
    """Same in FP32: per-step agreement to FP32 round-off relative to the solution scale."""
    sc = random_tiny(nx, ny, 500 + nx * 10 + ny)
    _print_case("tiny32", nx, ny)
    f = fl.from_scenario(sc, "f32", steps_per_graph=6)
    o = oracle.Run(sc)
    for step in range(12):
        f.step(1)
        o.step(1)
        h = f.get_depth()
        qx, qy = f.get_discharge()
        sh = max(np.abs(o.h).max(), 1e-3)
        sq = max(np.abs(o.qx).max(), np.abs(o.qy).max(), 1e-3)
        assert max_abs(h, o.h) <= 2e-5 * sh, (step, max_abs(h, o.h))
        assert max_abs(qx, o.qx) <= 2e-5 * sq, step
        assert max_abs(qy, o.qy) <= 2e-5 * sq, step
    f.close()


# -------------------------------------------------------------- the 256^2 valley
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_d1_valley_2000_steps(precision):
    """256^2 valley, dx 10 m, 100 m^3/s over 5 west cells, dry start, 2000 CFL steps."""
    sc = config_d1()
    _print_case("d1", precision)
    h, qx, qy, r = run_gpu(sc, sc.steps, precision)
    o = run_oracle(sc, sc.steps)
    assert r.steps == o.clock.steps == sc.steps
    if precision == "f64":
        assert rel_err(h, o.h) <= 1e-10
        assert rel_err(qx, o.qx) <= 1e-10
        assert rel_err(qy, o.qy) <= 1e-10
        assert abs(r.t - o.clock.t) <= 1e-10 * o.clock.t
        assert r.budget_error() <= 1e-12
    else:
        assert max_abs(h, o.h) <= 1e-3
        assert abs(r.t / o.clock.t - 1) <= 1e-5
        assert r.budget_error() <= 1e-6
    assert abs(r.v_in / o.clock.v_in - 1) <= (1e-10 if precision == "f64" else 1e-5)


# --------------------------------------------------------------- tiling invariance
def _ragged_valley(nx, ny, seed=9):
    from synth import Valley, manning_field, valley_dem64, west_section
    v = Valley(nx, ny, 5.0, 1e-3, 2.0, 30.0, 0.4, seed=seed, meander=True)
    z = valley_dem64(v).astype(np.float32)
    n = manning_field(v).astype(np.float32)
    first, count = west_section(v, 25.0)
    return Scenario(f"ragged_{nx}x{ny}", nx, ny, 5.0, z, n, np.zeros_like(z),
                    (WEST, first, count, 1e-3, np.array([0.0, 300.0]), np.array([30.0, 120.0])),
                    (EAST, 0, ny, 1e-3), dt_max=0.5)


def test_tiling_bitwise_invariance_and_parity():
    """A ragged 509 x 131 grid under every cells-per-lane and several rows-per-item:
    bit-identical states, and FP32 parity with the oracle."""
    sc = _ragged_valley(509, 131)
    ref = None
    for cpl in (1, 2, 4):
        for rows in (3, 16, 64, 256):
            _print_case("tiling", cpl, rows)
            h, qx, qy, r = run_gpu(sc, 400, "f32", cells_per_lane=cpl, rows_per_item=rows)
            if ref is None:
                ref = (h, qx, qy, r.t)
            else:
                assert np.array_equal(h, ref[0]), (cpl, rows)
                assert np.array_equal(qx, ref[1]) and np.array_equal(qy, ref[2]), (cpl, rows)
                assert r.t == ref[3]
    o = run_oracle(sc, 400)
    assert np.abs(o.h).max() > 0.1
    assert max_abs(ref[0], o.h) <= 1e-3


def test_tiling_fp64_parity():
    sc = _ragged_valley(301, 77, seed=4)
    o = run_oracle(sc, 300)
    for cpl, rows in ((1, 5), (2, 32)):
        _print_case("tiling64", cpl, rows)
        h, qx, qy, r = run_gpu(sc, 300, "f64", cells_per_lane=cpl, rows_per_item=rows)
        assert rel_err(h, o.h) <= 1e-10
        assert rel_err(qx, o.qx) <= 1e-10 and rel_err(qy, o.qy) <= 1e-10


# -------------------------------------------------------------- boundary sides
@pytest.mark.parametrize("side_in,side_out", [(WEST, EAST), (EAST, WEST), (SOUTH, NORTH),
                                              (NORTH, SOUTH), (WEST, SOUTH), (NORTH, EAST)])
def test_boundary_sides_fp64(side_in, side_out):
    """Inflow and outflow on every side: FP64 parity and the budget."""
    rng = np.random.default_rng(side_in * 4 + side_out)
    nx, ny = 70, 45
    z = rng.uniform(0.0, 0.5, (ny, nx)).astype(np.float32)
    n = rng.uniform(0.02, 0.06, (ny, nx)).astype(np.float32)
    L_in = ny if side_in in (WEST, EAST) else nx
    L_out = ny if side_out in (WEST, EAST) else nx
    sc = Scenario("sides", nx, ny, 2.0, z, n, np.zeros_like(z),
                  (side_in, L_in // 3, L_in // 3, 1e-3, np.array([0.0, 100.0]), np.array([5.0, 40.0])),
                  (side_out, 2, L_out - 4, 1e-3), dt_max=0.3)
    _print_case("sides", side_in, side_out)
    h, qx, qy, r = run_gpu(sc, 500, "f64", cells_per_lane=1, rows_per_item=16)
    o = run_oracle(sc, 500)
    assert np.abs(o.h).max() > 0.05
    assert rel_err(h, o.h) <= 1e-10
    assert rel_err(qx, o.qx) <= 1e-10 and rel_err(qy, o.qy) <= 1e-10
    assert r.budget_error() <= 1e-12
    if o.clock.v_out > 0:
        assert abs(r.v_out / o.clock.v_out - 1) <= 1e-10


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_lake_at_rest_bitwise_gpu(precision):
    """A flat water surface over a rough quantised bed stays bitwise still on the GPU."""
    rng = np.random.default_rng(17)
    nx, ny = 333, 97
    z = (np.round(rng.uniform(0.0, 3.0, (ny, nx)) * 256) / 256).astype(np.float32)
    h0 = np.maximum(np.float32(1.5) - z, np.float32(0)).astype(np.float32)
    sc = Scenario("lake", nx, ny, 2.0, z, rng.uniform(0.02, 0.08, (ny, nx)).astype(np.float32), h0,
                  None, None, dt_max=0.5)
    _print_case("lake", precision)
    h, qx, qy, r = run_gpu(sc, 3000, precision)
    assert np.array_equal(h, h0.astype(h.dtype))
    assert not qx.any() and not qy.any()
    assert r.steps == 3000


def test_closed_basin_volume_constant_gpu():
    sc = random_tiny(150, 90, 7, with_bc=False)
    sc.dx = 1.0
    _print_case("closed")
    f = fl.from_scenario(sc, "f64")
    f.step(300)
    r = f.get_report()
    assert abs(r.v_now / r.v0 - 1) <= 1e-13
    assert r.v_in == 0 and r.v_out == 0
    f.close()


@pytest.mark.parametrize("fusion", [1, 2])
def test_zero_threshold_thin_films_fp32(fusion):
    """h_eps = 0 with films down to 1e-30 m beside deep water and zero
    discharges: the FP32 face update (which multiplies by h_f^(-7/3)) stays
    finite and agrees with the oracle, and so does the donor factor of cells
    whose outflow is vanishingly small."""
    rng = np.random.default_rng(77)
    nx, ny = 48, 40
    z = rng.uniform(0.0, 0.5, (ny, nx)).astype(np.float32)
    n = rng.uniform(0.02, 0.06, (ny, nx)).astype(np.float32)
    kind = rng.random((ny, nx))
    h = np.where(kind < 0.4, 10.0 ** rng.uniform(-30, -18, (ny, nx)),
                 np.where(kind < 0.7, 0.0, rng.uniform(0.05, 1.0, (ny, nx)))).astype(np.float32)
    sc = Scenario("films", nx, ny, 1.0, z, n, h, None, None, dt_max=0.05, h_eps=0.0)
    f = fl.from_scenario(sc, "f32", fusion=fusion)
    o = oracle.Run(sc)
    for chunk in (2, 2, 4):
        f.step(chunk)
        o.step(chunk)
        hg = f.get_depth()
        qx, qy = f.get_discharge()
        assert np.isfinite(hg).all() and np.isfinite(qx).all() and np.isfinite(qy).all()
        sh = max(np.abs(o.h).max(), 1e-3)
        sq = max(np.abs(o.qx).max(), np.abs(o.qy).max(), 1e-3)
        assert max_abs(hg, o.h) <= 2e-5 * sh
        assert max_abs(qx, o.qx) <= 2e-5 * sq and max_abs(qy, o.qy) <= 2e-5 * sq
    r = f.get_report()
    assert r.nonfinite == 0 and r.budget_error() <= 1e-6
    f.close()
