"""Pins of the FP64 CPU adjoint: its gradients must equal central finite
differences of the FP64 forward run (the derivative's definition), for the
per-cell Manning n and every hydrograph sample, in a fully wet regime and in a
wet/dry regime where the donor-cell limiter is active."""
import numpy as np
import pytest

import oracle
from synth import EAST, WEST, Scenario

N, OBS_EVERY, NG = 200, 10, 12


def _scen(wet, seed=0, nx=16, ny=14):
    rng = np.random.default_rng(seed)
    dx, S = 5.0, 1e-3
    x = (np.arange(nx) + 0.5) * dx
    z = np.tile(S * (nx * dx - x), (ny, 1)) + rng.uniform(0, 0.05, (ny, nx))
    n = rng.uniform(0.03, 0.05, (ny, nx))
    if wet:
        h0 = np.maximum(1.2 - (z - z.min()), 0.3)
    else:
        h0 = np.where(rng.random((ny, nx)) < 0.5, rng.uniform(0, 0.02, (ny, nx)),
                      rng.uniform(0.2, 0.6, (ny, nx)))
    ts = np.linspace(0, 100, 6)
    qs = np.array([5.0, 8.0, 12.0, 9.0, 6.0, 5.0])
    return Scenario("adj", nx, ny, dx, z, n, h0, (WEST, 3, 6, S, ts, qs), (EAST, 0, ny, S),
                    dt_max=0.5, dt_fixed=0.5)


def _setup(wet):
    sc = _scen(wet)
    rng = np.random.default_rng(5)
    gauges = rng.choice(sc.nx * sc.ny, NG, replace=False)
    truth, _, _, _ = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=np.zeros((N // OBS_EVERY, NG)),
                                    n=sc.n * 1.1)
    return sc, gauges, truth


def _fd_check(sc, gauges, truth, tol):
    series, L, gn, gq = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=truth)
    assert L > 0

    def loss(n=None, qs=None):
        return oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=truth, n=n, qs=qs)[1]

    pairs = []
    rng = np.random.default_rng(8)
    side, first, count = sc.inflow[:3]
    inflow_cells = [(first + k) * sc.nx for k in (0, count // 2, count - 1)]   # west edge
    for c in list(rng.choice(sc.nx * sc.ny, 8, replace=False)) + inflow_cells:
        j, i = divmod(int(c), sc.nx)
        eps = 1e-6 * sc.n[j, i]
        p, m = sc.n.copy(), sc.n.copy()
        p[j, i] += eps
        m[j, i] -= eps
        pairs.append((gn[j, i], (loss(n=p) - loss(n=m)) / (2 * eps)))
    qs0 = sc.inflow[5]
    for k in range(len(qs0)):
        eps = 1e-6 * qs0[k]
        p, m = qs0.copy(), qs0.copy()
        p[k] += eps
        m[k] -= eps
        pairs.append((gq[k], (loss(qs=p) - loss(qs=m)) / (2 * eps)))
    scale = max(abs(f) for _, f in pairs)
    worst = max(abs(a - f) for a, f in pairs) / scale
    assert worst <= tol, worst
    return series, L, gn, gq


def test_adjoint_matches_finite_differences_wet():
    sc, gauges, truth = _setup(True)
    _fd_check(sc, gauges, truth, 1e-7)


def test_adjoint_matches_finite_differences_wet_dry_with_limiter():
    sc, gauges, truth = _setup(False)
    # the donor-cell limiter is active in this run: switching it off changes the loss
    l_on = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=truth)[1]
    l_off = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=truth, positivity=False)[1]
    assert abs(l_on - l_off) > 1e-6 * l_on
    _fd_check(sc, gauges, truth, 1e-5)


def test_adjoint_seeds_equal_squared_misfit():
    """Seeding with dL/dseries = 2 (series - obs) reproduces the squared-misfit gradient."""
    sc, gauges, truth = _setup(True)
    series, L, gn, gq = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=truth)
    _, _, gn2, gq2 = oracle.adjoint(sc, N, gauges, OBS_EVERY, dl_dseries=2 * (series - truth))
    assert np.allclose(gn, gn2, rtol=0, atol=1e-15 * np.abs(gn).max())
    assert np.allclose(gq, gq2, rtol=0, atol=1e-15 * np.abs(gq).max())
