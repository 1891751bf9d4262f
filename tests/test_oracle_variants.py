"""Pins of the oracle's two method variants (reading checks, off by default).

friction_vector: |q| in the friction term of eq. (3) is the magnitude of the
discharge vector at the face (the vector norm of eq. 2), the perpendicular
component averaged from the four perpendicular faces around the face.
boundary_cell_area: eq. (5)/(6) taken literally, A = dx^2 and the hydraulic
radius = the depth, so a boundary cell passes dx^2 h^{2/3} sqrt(S) / n.

As for the default readings, no test re-types the oracle's arithmetic: each
checks a reduction to the default, a closed form of the physics, a symmetry or
conservation, chosen so that a wrong face, index, factor or exponent in the
variant code fails one of them.
"""
import math

import numpy as np
import pytest

import oracle
from synth import EAST, NORTH, SOUTH, WEST, Scenario, config_d1


def _plane(nx, ny, dx, S):
    x = (np.arange(nx) + 0.5) * dx
    return np.tile(S * (nx * dx - x), (ny, 1))


def _normal_depth_case(nx=64, ny=4, dx=10.0, q=2.0, S=1e-3, nman=0.03):
    return Scenario("nd", nx, ny, dx, _plane(nx, ny, dx, S), np.full((ny, nx), nman),
                    np.full((ny, nx), 1.0),
                    (WEST, 0, ny, S, np.array([0.0]), np.array([q * ny * dx])), (EAST, 0, ny, S),
                    dt_max=2.0)


# ---------------------------------------------------------------- friction_vector
def test_vector_friction_without_cross_flow_is_the_face_form():
    """With no flow across the axis (qy = 0 everywhere, a 1-D channel) the
    vector magnitude is the face's own |q|: the run is bitwise the default."""
    sc = _normal_depth_case()
    a, b = oracle.Run(sc), oracle.Run(sc, friction_vector=True)
    a.step(3000)
    b.step(3000)
    assert not a.qy.any()
    assert np.array_equal(a.h, b.h) and np.array_equal(a.qx, b.qx) and np.array_equal(a.qy, b.qy)


def test_vector_friction_uniform_diagonal_flow_decay():
    """Uniform flow (qx, qy) = (a, b) over a flat bed of uniform depth H in a
    closed basin: away from the walls the surface stays flat and the depth
    constant, so each step is pure friction, the semi-implicit Manning law
    (qx, qy) <- (qx, qy) / (1 + g dt n^2 |q| / H^{7/3}) with |q| the magnitude
    of the vector.  The face (1-D) form would use |qx| and |qy| separately."""
    nx = ny = 40
    dx, H, nman, dt, a0, b0 = 5.0, 1.5, 0.08, 0.5, 0.6, -0.8
    qx0 = np.zeros((ny, nx + 1))
    qy0 = np.zeros((ny + 1, nx))
    qx0[:, 1:nx] = a0
    qy0[1:ny, :] = b0
    sc = Scenario("diag", nx, ny, dx, np.zeros((ny, nx)), np.full((ny, nx), nman),
                  np.full((ny, nx), H), None, None, dt_max=dt, dt_fixed=dt)
    sc.extra["qx0"], sc.extra["qy0"] = qx0, qy0
    steps = 5
    r = oracle.Run(sc, friction_vector=True)
    r.step(steps)
    d = oracle.Run(sc)
    d.step(steps)
    c = 9.81 * dt * nman ** 2 / H ** (7.0 / 3.0)
    qa, qb = a0, b0
    fa, fb = a0, b0          # the face form, for contrast
    for _ in range(steps):
        m = math.hypot(qa, qb)
        qa, qb = qa / (1 + c * m), qb / (1 + c * m)
        fa, fb = fa / (1 + c * abs(fa)), fb / (1 + c * abs(fb))
    cen = slice(14, 27)
    # first step: the surface is still flat everywhere, so faces along the
    # walls (whose perpendicular mean leaves the border faces out) decay like
    # the centre
    r1 = oracle.Run(sc, friction_vector=True)
    r1.step(1)
    assert np.array_equal(r1.qx[0, 2:nx - 1], r1.qx[ny // 2, 2:nx - 1])
    assert np.array_equal(r1.qx[ny - 1, 2:nx - 1], r1.qx[ny // 2, 2:nx - 1])
    assert np.array_equal(r1.qy[2:ny - 1, 0], r1.qy[2:ny - 1, nx // 2])
    assert np.array_equal(r1.qy[2:ny - 1, nx - 1], r1.qy[2:ny - 1, nx // 2])
    assert np.abs(r.h[cen, cen] - H).max() == 0.0
    assert np.abs(r.qx[cen, cen] / qa - 1).max() <= 1e-13
    assert np.abs(r.qy[cen, cen] / qb - 1).max() <= 1e-13
    assert np.abs(d.qx[cen, cen] / fa - 1).max() <= 1e-13
    assert abs(qa / fa - 1) > 1e-2         # the two readings differ here


def test_vector_friction_transpose_symmetry():
    """Transposing the problem (sides swapped) transposes the solution of the
    variant: the perpendicular mean treats both axes alike."""
    nx, ny, dx = 20, 14, 5.0
    rng = np.random.default_rng(5)
    z = _plane(nx, ny, dx, 2e-3) + rng.uniform(0, 0.3, (ny, nx))
    n = rng.uniform(0.02, 0.08, (ny, nx))
    hyd = (np.array([0.0, 40.0]), np.array([4.0, 25.0]))
    a = Scenario("a", nx, ny, dx, z, n, np.zeros((ny, nx)), (WEST, 3, 5, 2e-3, *hyd),
                 (EAST, 0, ny, 2e-3), dt_max=0.5)
    b = Scenario("b", ny, nx, dx, z.T.copy(), n.T.copy(), np.zeros((nx, ny)),
                 (SOUTH, 3, 5, 2e-3, *hyd), (NORTH, 0, ny, 2e-3), dt_max=0.5)
    ra, rb = oracle.Run(a, friction_vector=True), oracle.Run(b, friction_vector=True)
    ra.step(500)
    rb.step(500)
    s = ra.h.max()
    assert s > 0.05
    assert np.abs(ra.h - rb.h.T).max() <= 1e-11 * s
    qs = np.abs(ra.qx).max()
    assert np.abs(ra.qx - rb.qy.T).max() <= 1e-11 * qs
    assert np.abs(ra.qy - rb.qx.T).max() <= 1e-11 * qs
    # and the variant changed the result (cross flow exists here)
    d = oracle.Run(a)
    d.step(500)
    assert np.abs(d.h - ra.h).max() > 1e-6 * s


def test_vector_friction_mirror_symmetry_y():
    """A problem mirror-symmetric in y gives a mirror-symmetric solution with
    the variant: h and qx even, qy odd.  A perpendicular mean taken from the
    wrong rows (shifted by one) breaks this."""
    nx, ny, dx = 24, 10, 5.0
    rng = np.random.default_rng(11)
    half = rng.uniform(0, 0.4, (ny // 2, nx))
    z = _plane(nx, ny, dx, 2e-3) + np.concatenate([half, half[::-1]], axis=0)
    nh = rng.uniform(0.02, 0.08, (ny // 2, nx))
    n = np.concatenate([nh, nh[::-1]], axis=0)
    sc = Scenario("mirror", nx, ny, dx, z, n, np.zeros((ny, nx)),
                  (WEST, 2, 6, 2e-3, np.array([0.0, 50.0]), np.array([5.0, 30.0])),
                  (EAST, 0, ny, 2e-3), dt_max=0.5)
    r = oracle.Run(sc, friction_vector=True)
    r.step(600)
    s = r.h.max()
    assert s > 0.05
    assert np.abs(r.h - r.h[::-1]).max() <= 1e-11 * s
    qs = np.abs(r.qx).max()
    assert np.abs(r.qx - r.qx[::-1]).max() <= 1e-11 * qs
    assert np.abs(r.qy + r.qy[::-1]).max() <= 1e-11 * qs
    assert np.abs(r.qy).max() > 1e-3


def test_vector_friction_mass_budget():
    sc = config_d1()
    r = oracle.Run(sc, friction_vector=True)
    r.step(600)
    assert r.clock.v_in > 0 and r.budget_error() <= 1e-12


# ------------------------------------------------------------- boundary_cell_area
def test_cell_area_inflow_split_equal_bed():
    """Equal bed across the section: sum_c dx^2 k_c hhat^(2/3) = Q gives every cell
    the depth hhat = (Q / (dx^2 sum k))^(3/2); the faces carry Q in total."""
    rng = np.random.default_rng(3)
    nc, dx, S, Q = 9, 4.0, 2e-3, 137.0
    zc = np.full(nc, 12.25)
    nman = rng.uniform(0.02, 0.07, nc)
    kc = math.sqrt(S) / nman
    W, q = oracle.inflow_split_area(zc, kc, dx, Q)
    hhat = (Q / (dx * dx * kc.sum())) ** 1.5
    assert abs((W - 12.25) / hhat - 1) <= 1e-12
    assert abs(dx * q.sum() / Q - 1) <= 1e-13
    # per-unit-width face discharge of a cell: dx k hhat^(2/3)
    assert np.abs(q / (dx * kc * hhat ** (2.0 / 3.0)) - 1).max() <= 1e-12
    # the default reading gives another depth for the same Q
    W5, _ = oracle.inflow_split(zc, kc, dx, Q)
    assert abs((W5 - 12.25) / hhat - 1) > 1e-2


def test_cell_area_inflow_split_uneven_bed():
    rng = np.random.default_rng(8)
    zc = rng.uniform(0.0, 2.0, 15)
    kc = math.sqrt(1e-3) / rng.uniform(0.02, 0.07, 15)
    for Q in (0.5, 20.0, 900.0):
        W, q = oracle.inflow_split_area(zc, kc, 3.0, Q)
        assert abs(3.0 * q.sum() / Q - 1) <= 1e-12
        assert np.all(q[zc >= W] == 0) and np.all(q[zc < W] > 0)


def test_cell_area_outflow_steady_edge_depth():
    """A short channel on a plane with the literal boundaries converges to a
    steady state with q = Q / width on every x-face; the outflow cell then
    holds the depth at which dx h^(2/3) sqrt(S) / n = q, i.e.
    h_e = (q n / (dx sqrt S))^(3/2) -- not the interior's normal depth."""
    nx, ny, dx, q, S, nman = 20, 3, 2.0, 4.0, 1e-3, 0.05
    sc = Scenario("ca", nx, ny, dx, _plane(nx, ny, dx, S), np.full((ny, nx), nman),
                  np.full((ny, nx), 4.0),
                  (WEST, 0, ny, S, np.array([0.0]), np.array([q * ny * dx])), (EAST, 0, ny, S),
                  dt_max=2.0)
    r = oracle.Run(sc, boundary_cell_area=True, nthreads=1)
    r.step(40000)
    h_e = (q * nman / (dx * math.sqrt(S))) ** 1.5
    h_n = (q * nman / math.sqrt(S)) ** 0.6
    assert abs(h_e / h_n - 1) > 0.5         # the literal outlet differs from the normal depth
    assert np.abs(r.h[:, -1] / h_e - 1).max() <= 1e-6
    assert np.abs(r.qx / q - 1).max() <= 1e-6
    assert np.abs(r.qy).max() <= 1e-9


def test_cell_area_mass_budget():
    sc = config_d1()
    r = oracle.Run(sc, boundary_cell_area=True)
    r.step(600)
    assert r.clock.v_in > 0 and r.clock.v_out >= 0 and r.budget_error() <= 1e-12

