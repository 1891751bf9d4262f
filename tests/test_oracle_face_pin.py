"""Single-face pins of the oracle: one step on a 2x1 (and 1x2) grid worked out by hand.

Eq. (3) (with the dt of reading R1 on the gravity term), eq. (4) and the donor
scaling of reading R7 on the one interior face of a two-cell grid with closed
walls, g = 9.81, dx = 1 m, a fixed dt = 0.1 s (so g*dt = 0.981).  Each expected
value below was worked out by hand from the equations and is written as a
number, so that a slip in the oracle's face update (a dropped term, a wrong
exponent, sign, mean or depth of the face) is caught by arithmetic done
independently of it.
"""
import numpy as np
import pytest

import oracle
from synth import Scenario

DT = 0.1


def _one_step(h, z, n, q0=0.0, axis="x"):
    """Two cells along `axis`; returns (h after one step, interior face discharge)."""
    h = np.asarray(h, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    if axis == "x":
        shape, nx, ny = (1, 2), 2, 1
        extra = {"qx0": np.array([[0.0, q0, 0.0]])}
    else:
        shape, nx, ny = (2, 1), 1, 2
        extra = {"qy0": np.array([[0.0], [q0], [0.0]])}
    sc = Scenario("face", nx, ny, 1.0, z.reshape(shape), n.reshape(shape), h.reshape(shape),
                  None, None, dt_max=DT, dt_fixed=DT, extra=extra)
    r = oracle.Run(sc)
    assert r.step(1) == 0
    assert r.clock.steps == 1 and r.clock.t == pytest.approx(DT, rel=0, abs=1e-15)
    # the walls stay closed
    if axis == "x":
        assert r.qx[0, 0] == 0.0 and r.qx[0, 2] == 0.0 and not r.qy.any()
        return r.h.reshape(-1), r.qx[0, 1]
    assert r.qy[0, 0] == 0.0 and r.qy[2, 0] == 0.0 and not r.qx.any()
    return r.h.reshape(-1), r.qy[1, 0]


def _close(a, b, rel=1e-13):
    return abs(a - b) <= rel * max(abs(b), 1e-300)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_gravity_term_still_water(axis):
    """h = (2, 1) on a flat bed, q = 0: h_f = 2, slope -1, so q = 0.981*2 = 1.962 and
    0.1962 m moves from the first cell to the second (no friction at q = 0)."""
    h, q = _one_step([2.0, 1.0], [0.0, 0.0], [0.05, 0.05], axis=axis)
    assert _close(q, 1.962)
    assert _close(h[0], 1.8038) and _close(h[1], 1.1962)
    # mirrored: the same flow the other way
    h, q = _one_step([1.0, 2.0], [0.0, 0.0], [0.05, 0.05], axis=axis)
    assert _close(q, -1.962)
    assert _close(h[0], 1.1962) and _close(h[1], 1.8038)


def test_face_depth_is_surface_above_higher_bed():
    """Bed (0.5, 0), depth (1, 1): surfaces 1.5 and 1, face depth 1.5 - 0.5 = 1,
    slope -0.5, so q = 0.981*1*0.5 = 0.4905 (reading R3; the deeper-cell depth 1 gives
    the same here, the surface above the lower bed would give 0.73575)."""
    h, q = _one_step([1.0, 1.0], [0.5, 0.0], [0.03, 0.03])
    assert _close(q, 0.4905)
    assert _close(h[0], 0.95095) and _close(h[1], 1.04905)
    # deeper water on the higher bed: depths (1, 2), beds (1, 0): surfaces 2 and 2, no flow
    h, q = _one_step([1.0, 2.0], [1.0, 0.0], [0.03, 0.03])
    assert q == 0.0 and h[0] == 1.0 and h[1] == 2.0


def test_friction_with_flat_surface():
    """Flat surface (depths 1, 1), q = 2, n = 0.1: the gravity term vanishes and
    q' = 2 / (1 + 0.981*0.01*2/1) = 2/1.01962."""
    h, q = _one_step([1.0, 1.0], [0.0, 0.0], [0.1, 0.1], q0=2.0)
    assert _close(q, 2.0 / 1.01962)
    assert _close(h[0], 1.0 - 0.2 / 1.01962) and _close(h[1], 1.0 + 0.2 / 1.01962)
    # the face's n is the mean of the two cells' n: (0.1 + 0.3)/2 = 0.2, n^2 = 0.04
    h, q = _one_step([1.0, 1.0], [0.0, 0.0], [0.1, 0.3], q0=2.0, axis="y")
    assert _close(q, 2.0 / 1.07848)


def test_friction_depth_exponent():
    """Face depth 8: h_f^(7/3) = 128, so q' = 2 / (1 + 0.01962/128) = 2/1.00015328125."""
    h, q = _one_step([8.0, 8.0], [0.0, 0.0], [0.1, 0.1], q0=2.0)
    assert _close(q, 2.0 / 1.00015328125)
    # backward flow: |q| in the friction term, the sign kept
    h, q = _one_step([8.0, 8.0], [0.0, 0.0], [0.1, 0.1], q0=-2.0)
    assert _close(q, -2.0 / 1.00015328125)


def test_dry_face_below_threshold():
    """Face depth 5e-5 m <= h_eps = 1e-4 m: the face carries nothing, even with a slope
    and an incoming discharge."""
    h, q = _one_step([5e-5, 0.0], [0.0, 0.0], [0.03, 0.03], q0=0.5)
    assert q == 0.0 and h[0] == 5e-5 and h[1] == 0.0


def test_donor_scaling_drains_exactly():
    """Depths (0.01, 0.01), flat surface, n = 0, q = 1: eq. (3) keeps q* = 1, which
    would take 0.1 m from a cell holding 0.01 m.  The donor factor 0.01/0.1 = 0.1
    applies q = 0.1: the first cell empties exactly and the second holds 0.02 m."""
    h, q = _one_step([0.01, 0.01], [0.0, 0.0], [0.0, 0.0], q0=1.0)
    assert _close(q, 0.1)
    assert abs(h[0]) <= 1e-17 and _close(h[1], 0.02)
