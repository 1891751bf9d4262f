"""Reverse mode at its full configuration: the 1024^2 valley at dx 5 m, fixed
dt 0.25 s (the paper's constant-step mode), 5000 steps with ceil(sqrt(N)) = 71
checkpoints, a 100-sample inflow hydrograph, and the squared depth misfit at
500 gauges (wet cells of a truth run with perturbed roughness) observed every
50 steps.

* FP64 GPU gradients against central differences of the FP64 GPU forward,
  for 16 wet cells' Manning n and 8 hydrograph samples.  The loss is only
  piecewise smooth in the parameters (the max() of the face depth, the donor
  limiter, |q|, dry faces, the front advancing over dry cells): with a
  relative step of 1e-4 the differences of the early hydrograph samples cross
  kinks and land 1.5e-3 off the adjoint, and they converge onto it as the step
  shrinks (measured on this configuration, with h_eps 1e-4 and 0 alike: at
  1e-6 the cells are within 6e-6 and the samples within 1.1e-4).  The steps
  are therefore 1e-6 of a cell's n and 1e-7 of a sample's Q.  FP64 rounding of
  the loss (~1e-13) then leaves ~2e-6 absolute noise in a cell's difference
  quotient and ~1e-9 in a sample's; the compared parameters carry gradients of
  at least 1e-2 of the largest (>= 0.1 for cells), so the noise stays well
  below the 1e-4 gate.
* FP32 GPU gradients against the FP64 GPU gradients over every cell's n and
  every hydrograph sample: relative L2 <= 1e-2 and cosine >= 0.999.
"""
import numpy as np
import pytest

import paper_2204_10323_amd as fl
import synth
from synth import Scenario

pytestmark = pytest.mark.gpu

STEPS, OBS_EVERY, NGAUGES = 5000, 50, 500
EPS_N, EPS_Q = 1e-6, 1e-7   # relative central-difference steps
# FD against the adjoint: |fd - adj| <= FD_TOL * |adj|, for parameters whose
# gradient is at least FD_FLOOR of the largest
FD_TOL, FD_FLOOR = 1e-4, 1e-2


def _with(sc, n=None, qs=None):
    side, first, count, slope, ts, q0 = sc.inflow
    return Scenario(sc.name, sc.nx, sc.ny, sc.dx, sc.z, sc.n if n is None else n, sc.h0,
                    (side, first, count, slope, ts, q0 if qs is None else qs), sc.outflow,
                    dt_max=sc.dt_max, dt_fixed=sc.dt_fixed)


def _loss(sc, gauges, obs, n=None, qs=None):
    f = fl.from_scenario(_with(sc, n, qs), "f64")
    f.adj_setup(gauges, OBS_EVERY, obs)
    _, loss = f.adj_forward(STEPS)
    f.close()
    return loss


def _grads(sc, prec, gauges, obs):
    f = fl.from_scenario(sc, prec)
    f.adj_setup(gauges, OBS_EVERY, obs.astype(f.dtype))
    _, loss = f.adj_forward(STEPS)
    gn, gq = f.adj_backward(None, len(sc.inflow[5]))
    f.close()
    return loss, gn, gq


@pytest.fixture(scope="module")
def problem():
    sc = synth.config_d5(1024, STEPS)
    truth = _with(sc, n=sc.extra["n_true"])
    print("CASE adjoint gate: FP64 truth run", flush=True)
    t = fl.from_scenario(truth, "f64")
    t.step(STEPS)
    h_end = t.get_depth()
    t.close()
    rng = np.random.default_rng(55)
    gauges = rng.choice(np.nonzero(h_end.ravel() > 0.05)[0], NGAUGES, replace=False)
    t = fl.from_scenario(truth, "f64")
    t.adj_setup(gauges, OBS_EVERY)
    obs, _ = t.adj_forward(STEPS)
    t.close()
    print("CASE adjoint gate: FP64 forward + reverse", flush=True)
    loss, gn, gq = _grads(sc, "f64", gauges, obs)
    return sc, gauges, obs, loss, gn, gq


def test_fp64_gradients_against_central_differences(problem):
    sc, gauges, obs, loss, gn, gq = problem
    assert loss > 0 and np.isfinite(gn).all() and np.isfinite(gq).all()
    rng = np.random.default_rng(7)
    flat = np.abs(gn).ravel()
    top = np.argsort(flat)[::-1]
    strong = rng.choice(top[:200], 8, replace=False)
    rest = np.nonzero(flat > FD_FLOOR * flat.max())[0]
    rest = rest[~np.isin(rest, strong)]
    cells = np.concatenate([strong, rng.choice(rest, 8, replace=False)])
    n64 = sc.n.astype(np.float64)
    worst = 0.0
    for c in cells:
        j, i = divmod(int(c), sc.nx)
        d = EPS_N * n64[j, i]
        lp = _loss(sc, gauges, obs, n=_bump(n64, j, i, d))
        lm = _loss(sc, gauges, obs, n=_bump(n64, j, i, -d))
        fd = (lp - lm) / (2 * d)
        ad = float(gn[j, i])
        rel = abs(fd - ad) / abs(ad)
        worst = max(worst, rel)
        print(f"n at ({j},{i}): adjoint {ad:.9e} fd {fd:.9e} rel {rel:.2e}", flush=True)
        assert rel <= FD_TOL
    qs = np.asarray(sc.inflow[5], dtype=np.float64)
    aq = np.abs(gq)
    ks = list(np.argsort(aq)[::-1][:4])
    others = [k for k in np.nonzero(aq > FD_FLOOR * aq.max())[0] if k not in ks]
    ks += list(rng.choice(others, 4, replace=False))
    for k in ks:
        d = EPS_Q * qs[k]
        qp, qm = qs.copy(), qs.copy()
        qp[k] += d
        qm[k] -= d
        fd = (_loss(sc, gauges, obs, qs=qp) - _loss(sc, gauges, obs, qs=qm)) / (2 * d)
        ad = float(gq[k])
        rel = abs(fd - ad) / abs(ad)
        worst = max(worst, rel)
        print(f"Q sample {k}: adjoint {ad:.9e} fd {fd:.9e} rel {rel:.2e}", flush=True)
        assert rel <= FD_TOL
    print(f"worst relative FD difference {worst:.2e}", flush=True)


def _bump(a, j, i, d):
    b = a.copy()
    b[j, i] += d
    return b


def _rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _cos(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_fp32_gradients_against_fp64(problem):
    sc, gauges, obs, loss, gn, gq = problem
    print("CASE adjoint gate: FP32 forward + reverse", flush=True)
    loss32, gn32, gq32 = _grads(sc, "f32", gauges, obs)
    rn, cn = _rel_l2(gn32, gn), _cos(gn32, gn)
    rq, cq = _rel_l2(gq32, gq), _cos(gq32, gq)
    print(f"loss fp32 {loss32:.9e} fp64 {loss:.9e}; grad_n rel L2 {rn:.2e} cos {cn:.6f}; "
          f"grad_q rel L2 {rq:.2e} cos {cq:.6f}", flush=True)
    assert abs(loss32 / loss - 1) <= 1e-2
    assert rn <= 1e-2 and cn >= 0.999
    assert rq <= 1e-2 and cq >= 0.999
