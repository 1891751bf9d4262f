"""Pins of the FP64 CPU oracle against facts fixed by the paper and by physics.

None of these tests re-types the oracle's formulas: each checks an invariant,
a textbook closed form or a symmetry that a plausible slip in the oracle (a
dropped dt, a wrong sign, exponent or index, a transposed operand, a
non-conservative update) would break.
"""
import math

import numpy as np
import pytest

import oracle
from synth import EAST, NORTH, SOUTH, WEST, Scenario, config_d1


def _plane(nx, ny, dx, S):
    x = (np.arange(nx) + 0.5) * dx
    return np.tile(S * (nx * dx - x), (ny, 1))


# ---------------------------------------------------------------- lake at rest
@pytest.mark.parametrize("fixed_dt", [0.0, 0.3])
def test_lake_at_rest_bitwise(fixed_dt):
    """A flat water surface over a rough bed stays exactly still (eq. 3 with h_f).

    Bed and surface are multiples of 2^-8 below 2^13 so h = eta - z and h + z
    are exact; wet/dry contact faces have h_f = 0.  Pins the h_f definition
    (max surface minus max bed), the gravity term and the depth update.
    """
    rng = np.random.default_rng(7)
    nx, ny = 37, 29
    z = np.round(rng.uniform(0.0, 3.0, (ny, nx)) * 256) / 256
    eta0 = 1.5
    h0 = np.maximum(eta0 - z, 0.0)
    assert (h0 > 0).any() and (h0 == 0).any()
    sc = Scenario("lake", nx, ny, 2.0, z, rng.uniform(0.02, 0.08, (ny, nx)), h0, None, None,
                  dt_max=0.5, dt_fixed=fixed_dt)
    r = oracle.Run(sc)
    assert r.step(10000) == 0
    assert r.clock.steps == 10000
    assert np.array_equal(r.h, h0)
    assert not r.qx.any() and not r.qy.any()


# ------------------------------------------------------------ mass conservation
def test_mass_budget_d1():
    """Volume = initial + inflow - outflow to round-off on the 256^2 valley (2000 steps)."""
    sc = config_d1()
    r = oracle.Run(sc)
    assert r.step(sc.steps) == 0
    assert r.clock.v_in > 0 and r.clock.v_out >= 0
    assert r.budget_error() <= 1e-12
    assert r.h.min() >= -1e-12 * r.h.max()


@pytest.mark.parametrize("seed", range(6))
def test_mass_budget_random(seed):
    """Random wet/dry states and boundary sections: the budget closes to 1e-12."""
    from synth import random_tiny
    rng = np.random.default_rng(seed)
    sc = random_tiny(int(rng.integers(3, 12)), int(rng.integers(3, 12)), seed)
    r = oracle.Run(sc)
    assert r.step(300) == 0
    assert r.budget_error() <= 1e-12


def test_closed_basin_volume_constant():
    """With every border closed the volume never changes (interior fluxes cancel)."""
    from synth import random_tiny
    sc = random_tiny(9, 7, 3, with_bc=False)
    r = oracle.Run(sc)
    v0 = r.volume()
    r.step(500)
    assert abs(r.volume() - v0) <= 1e-13 * v0
    assert r.clock.v_in == 0 and r.clock.v_out == 0


# ---------------------------------------------------- positivity (donor scaling)
def test_positivity_dam_break_onto_dry_bed():
    """A dam break onto a dry sloping bed keeps depths non-negative and conserves volume.

    The same run without donor scaling goes negative, which shows the scaling is
    what keeps the depths valid here.
    """
    nx, ny, dx = 40, 6, 1.0
    z = _plane(nx, ny, dx, 0.05)
    h0 = np.zeros((ny, nx))
    h0[:, :8] = 2.0
    sc = Scenario("dam", nx, ny, dx, z, np.full((ny, nx), 0.02), h0, None, (EAST, 0, ny, 0.05),
                  dt_max=1.0, alpha=0.9)
    r = oracle.Run(sc)
    worst = 0.0
    for _ in range(200):
        r.step(1)
        worst = min(worst, r.h.min())
    assert worst >= -1e-12
    assert r.budget_error() <= 1e-12
    r2 = oracle.Run(sc, positivity=False)
    worst2 = 0.0
    for _ in range(200):
        r2.step(1)
        worst2 = min(worst2, r2.h.min())
    assert worst2 < -1e-6


# ------------------------------------------------------ Manning normal depth
@pytest.mark.parametrize("q,S,nman", [(2.0, 1e-3, 0.03), (0.5, 5e-4, 0.05)])
def test_manning_normal_depth(q, S, nman):
    """Uniform flow on a plane converges to the textbook normal depth (q n / sqrt S)^(3/5).

    Inflow across the whole west edge and outflow across the whole east edge
    with the bed slope.  Pins the dt in eq. (3), the exponents 7/3 and 5/3, the
    face-section reading of A in eq. (5) and the boundary/interior agreement.
    """
    nx, ny, dx = 64, 4, 10.0
    hn = (q * nman / math.sqrt(S)) ** 0.6
    if q == 2.0:
        assert abs(hn - 1.4686) < 1e-4
    sc = Scenario("nd", nx, ny, dx, _plane(nx, ny, dx, S), np.full((ny, nx), nman),
                  np.full((ny, nx), 1.0),
                  (WEST, 0, ny, S, np.array([0.0]), np.array([q * ny * dx])), (EAST, 0, ny, S),
                  dt_max=2.0)
    r = oracle.Run(sc)
    r.step(20000)
    assert np.abs(r.h / hn - 1).max() <= 1e-6
    assert np.abs(r.qx / q - 1).max() <= 1e-6
    assert np.abs(r.qy).max() <= 1e-9


# ---------------------------------------------------------------- inflow split
def test_inflow_split_equal_bed():
    """Equal bed across the section: every cell gets depth (Q/(dx sum k))^(3/5) (eq. 6)."""
    rng = np.random.default_rng(3)
    nc, dx, S, Q = 9, 4.0, 2e-3, 137.0
    zc = np.full(nc, 12.25)
    nman = rng.uniform(0.02, 0.07, nc)
    kc = math.sqrt(S) / nman
    W, q = oracle.inflow_split(zc, kc, dx, Q)
    hhat = (Q / (dx * kc.sum())) ** 0.6
    assert abs((W - zc[0]) / hhat - 1) <= 1e-12
    assert abs(q.sum() * dx / Q - 1) <= 1e-12
    # equal roughness as well: the wide-section normal depth (Q n / (N dx sqrt S))^(3/5)
    W2, q2 = oracle.inflow_split(zc, np.full(nc, math.sqrt(S) / 0.03), dx, Q)
    assert abs((W2 - zc[0]) / (Q * 0.03 / (nc * dx * math.sqrt(S))) ** 0.6 - 1) <= 1e-12


def test_inflow_split_uneven_bed():
    """Uneven bed: the section carries exactly Q, dry cells above W carry nothing,
    and the deeper the cell the larger its discharge."""
    zc = np.array([3.0, 1.0, 0.5, 0.7, 2.0, 9.0])
    kc = np.full(6, 1.0)
    W, q = oracle.inflow_split(zc, kc, 5.0, 40.0)
    assert abs(q.sum() * 5.0 / 40.0 - 1) <= 1e-12
    assert q[5] == 0.0 and W < 9.0
    order = np.argsort(zc[:5])
    assert np.all(np.diff(q[:5][order]) < 0)


def test_hydrograph_interpolation():
    """Piecewise linear between samples, constant outside them."""
    ts, qs = np.array([0.0, 10.0, 30.0]), np.array([5.0, 25.0, 15.0])
    assert oracle.hydrograph(ts, qs, -3.0) == 5.0
    assert oracle.hydrograph(ts, qs, 5.0) == 15.0
    assert oracle.hydrograph(ts, qs, 20.0) == 20.0
    assert oracle.hydrograph(ts, qs, 99.0) == 15.0


# ---------------------------------------------------------------------- seiche
def test_seiche_period():
    """Linear gravity wave in a closed frictionless basin: period 2L/sqrt(gH) within 1%.

    dt = 0.5 s, so a missing dt in the gravity term of eq. (3) would change the
    period by sqrt(2); a wrong sign makes the mode grow instead of oscillate.
    """
    nx, dx, H, eps = 64, 10.0, 1.0, 1e-3
    L = nx * dx
    x = (np.arange(nx) + 0.5) * dx
    h0 = (H + eps * np.cos(np.pi * x / L))[None, :]
    sc = Scenario("seiche", nx, 1, dx, np.zeros((1, nx)), np.full((1, nx), 1e-4), h0, None, None,
                  dt_max=0.5, dt_fixed=0.5)
    r = oracle.Run(sc)
    T = 2 * L / math.sqrt(9.81 * H)
    sig, ts = [], []
    for k in range(int(3 * T / 0.5) + 1):
        r.step(1)
        sig.append(r.h[0, 0] - H)
        ts.append(r.clock.t)
    sig, ts = np.array(sig), np.array(ts)
    assert np.abs(sig).max() < 1.5 * eps
    cross = []
    for k in range(1, len(sig)):
        if sig[k - 1] > 0 >= sig[k] or sig[k - 1] < 0 <= sig[k]:
            cross.append(ts[k - 1] + (ts[k] - ts[k - 1]) * sig[k - 1] / (sig[k - 1] - sig[k]))
    period = 2 * np.mean(np.diff(cross))
    assert abs(period / T - 1) < 0.01


# -------------------------------------------------------------------- symmetry
def _sym_dem(nx, ny, dx, seed):
    rng = np.random.default_rng(seed)
    half = rng.uniform(0, 0.4, (ny // 2, nx))
    bumps = np.concatenate([half, half[::-1]], axis=0)
    return _plane(nx, ny, dx, 2e-3) + bumps


def test_mirror_symmetry_y():
    """A DEM, roughness and inflow section mirror-symmetric in y give a mirror-symmetric
    solution: h and qx even, qy odd.  Catches one-sided face roughness and index slips."""
    nx, ny, dx = 24, 10, 5.0
    z = _sym_dem(nx, ny, dx, 11)
    rng = np.random.default_rng(12)
    nh = rng.uniform(0.02, 0.08, (ny // 2, nx))
    n = np.concatenate([nh, nh[::-1]], axis=0)
    sc = Scenario("mirror", nx, ny, dx, z, n, np.zeros((ny, nx)),
                  (WEST, 2, 6, 2e-3, np.array([0.0, 50.0]), np.array([5.0, 30.0])),
                  (EAST, 0, ny, 2e-3), dt_max=0.5)
    r = oracle.Run(sc)
    r.step(600)
    assert r.h.max() > 0.05
    s = r.h.max()
    assert np.abs(r.h - r.h[::-1]).max() <= 1e-11 * s
    qs = np.abs(r.qx).max()
    assert np.abs(r.qx - r.qx[::-1]).max() <= 1e-11 * qs
    assert np.abs(r.qy + r.qy[::-1]).max() <= 1e-11 * qs
    assert np.abs(r.qy).max() > 1e-3


def test_transpose_symmetry():
    """Transposing the DEM and swapping west<->south, east<->north transposes the
    solution (qx <-> qy^T).  Catches a transposed operand or an x/y slip."""
    nx, ny, dx = 20, 14, 5.0
    rng = np.random.default_rng(5)
    z = _plane(nx, ny, dx, 2e-3) + rng.uniform(0, 0.3, (ny, nx))
    n = rng.uniform(0.02, 0.08, (ny, nx))
    hyd = (np.array([0.0, 40.0]), np.array([4.0, 25.0]))
    a = Scenario("a", nx, ny, dx, z, n, np.zeros((ny, nx)), (WEST, 3, 5, 2e-3, *hyd),
                 (EAST, 0, ny, 2e-3), dt_max=0.5)
    b = Scenario("b", ny, nx, dx, z.T.copy(), n.T.copy(), np.zeros((nx, ny)),
                 (SOUTH, 3, 5, 2e-3, *hyd), (NORTH, 0, ny, 2e-3), dt_max=0.5)
    ra, rb = oracle.Run(a), oracle.Run(b)
    ra.step(500)
    rb.step(500)
    s = ra.h.max()
    assert s > 0.05
    assert np.abs(ra.h - rb.h.T).max() <= 1e-11 * s
    qs = np.abs(ra.qx).max()
    assert np.abs(ra.qx - rb.qy.T).max() <= 1e-11 * qs
    assert np.abs(ra.qy - rb.qx.T).max() <= 1e-11 * qs


# ------------------------------------------------------------------ clock (CFL)
def test_cfl_clock_and_final_step():
    """Lake at rest on a flat bed of depth H: every CFL step is alpha dx / sqrt(g H),
    capped by dt_max, and the last step is shortened to land exactly on t_end."""
    nx, ny, dx, H, alpha = 8, 5, 3.0, 2.0, 0.7
    sc = Scenario("clock", nx, ny, dx, np.zeros((ny, nx)), np.full((ny, nx), 0.03),
                  np.full((ny, nx), H), None, None, dt_max=10.0, alpha=alpha, t_end=10.0)
    r = oracle.Run(sc)
    r.step(1)
    dt = alpha * dx / math.sqrt(9.81 * H)
    assert abs(r.clock.last_dt / dt - 1) < 1e-15
    nfull = math.ceil(10.0 / dt) - 1
    r.step(nfull - 1)
    t_prev = r.clock.t
    assert abs(t_prev / (nfull * dt) - 1) < 1e-13 and r.clock.done == 0
    r.step(1000)
    assert r.clock.done == 1 and r.clock.t == 10.0
    assert r.clock.steps == nfull + 1
    assert abs(r.clock.last_dt - (10.0 - t_prev)) < 1e-12 and r.clock.last_dt < 0.9 * dt
    n_before = r.clock.steps
    r.step(5)
    assert r.clock.steps == n_before
    sc2 = Scenario("cap", nx, ny, dx, np.zeros((ny, nx)), np.full((ny, nx), 0.03),
                   np.full((ny, nx), H), None, None, dt_max=0.25, alpha=alpha)
    r2 = oracle.Run(sc2)
    r2.step(3)
    assert r2.clock.last_dt == 0.25 and r2.clock.t == 0.75


def test_nonfinite_depth_is_reported():
    from synth import random_tiny
    sc = random_tiny(5, 4, 1)
    sc.h0 = sc.h0.copy()
    sc.h0[2, 3] = np.nan
    r = oracle.Run(sc)
    assert r.step(3) == 2 and r.clock.done == 2 and r.clock.steps == 0
