"""The GPU reverse mode (hand-written adjoint kernels, sqrt(N) checkpoints)
against the FP64 CPU adjoint and finite differences.

Gates (project-set; the method's build gives no number for the adjoint):
FP64 GPU vs FP64 CPU adjoint <= 1e-8 relative L2; FP32 GPU vs FP64 CPU <= 1e-2
relative L2 with cosine >= 0.999; FP64 GPU vs central differences of the FP64
GPU forward <= 1e-6 relative.
"""
import numpy as np
import pytest

import oracle
import paper_2204_10323_amd as fl
from synth import EAST, NORTH, SOUTH, WEST, Scenario, Valley, manning_field, valley_dem64

pytestmark = pytest.mark.gpu

N, OBS_EVERY, NG = 200, 10, 12


def _pin_scen(wet, seed=0, nx=16, ny=14):
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


def _valley_scen(nx=200, ny=150, seed=21):
    v = Valley(nx, ny, 5.0, 1e-3, 2.0, 30.0, 0.3, seed=seed, meander=True)
    z = valley_dem64(v)
    n = manning_field(v)
    h0 = np.maximum(np.percentile(z, 25) - z, 0.0)
    from synth import west_section
    first, count = west_section(v, 30.0)
    ts = np.linspace(0, 300, 11)
    qs = 20 + 15 * np.sin(ts / 50.0) ** 2
    return Scenario("valley_adj", nx, ny, 5.0, z, n, h0, (WEST, first, count, 1e-3, ts, qs),
                    (EAST, 0, ny, 1e-3), dt_max=0.5, dt_fixed=0.5)


def _cast(sc, dtype):
    return Scenario(sc.name, sc.nx, sc.ny, sc.dx, sc.z.astype(dtype), sc.n.astype(dtype),
                    sc.h0.astype(dtype), sc.inflow, sc.outflow, dt_max=sc.dt_max,
                    dt_fixed=sc.dt_fixed)


def _gpu_adjoint(sc, precision, gauges, obs, nsteps=N, ckpt=0, obs_every=OBS_EVERY):
    f = fl.from_scenario(sc, precision)
    f.adj_setup(gauges, obs_every, obs.astype(f.dtype), ckpt)
    series, loss = f.adj_forward(nsteps)
    gn, gq = f.adj_backward(None, len(sc.inflow[5]))
    return f, series, loss, gn, gq


def _rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.mark.parametrize("wet", [True, False])
def test_fp64_gpu_adjoint_matches_cpu_adjoint(wet):
    sc = _cast(_pin_scen(wet), np.float64)
    rng = np.random.default_rng(5)
    gauges = rng.choice(sc.nx * sc.ny, NG, replace=False)
    truth, _, _, _ = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=np.zeros((N // OBS_EVERY, NG)),
                                    n=sc.n * 1.1)
    s_cpu, l_cpu, gn_cpu, gq_cpu = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=truth)
    print("CASE adjoint fp64 wet=%s" % wet, flush=True)
    ref = None
    for ckpt in (0, 1, 7, N):
        f, s, l, gn, gq = _gpu_adjoint(sc, "f64", gauges, truth, ckpt=ckpt)
        f.close()
        assert np.abs(s - s_cpu).max() <= 1e-11 * max(1.0, np.abs(s_cpu).max())
        assert abs(l / l_cpu - 1) <= 1e-8
        assert _rel_l2(gn, gn_cpu) <= 1e-8, _rel_l2(gn, gn_cpu)
        assert _rel_l2(gq, gq_cpu) <= 1e-8, _rel_l2(gq, gq_cpu)
        if ref is None:
            ref = (gn, gq)
        else:   # the checkpoint stride changes nothing
            assert np.array_equal(gn, ref[0]) and np.array_equal(gq, ref[1])


@pytest.mark.parametrize("sides", [(EAST, WEST), (SOUTH, NORTH), (NORTH, SOUTH), (WEST, SOUTH)],
                         ids=["east_in_west_out", "south_in_north_out", "north_in_south_out",
                              "west_in_south_out"])
def test_fp64_gpu_adjoint_sections_on_every_side(sides):
    """Inflow and outflow sections on every side of a 71 x 23 grid (two strips of
    the reverse pass, chunks of a few rows): the reverse pass takes a west or
    east border by row and a south or north one by column, and writes the
    inflow adjoints from the row or column on the section."""
    in_side, out_side = sides
    nx, ny, dx, S = 71, 23, 5.0, 1e-3
    rng = np.random.default_rng(17)
    z = rng.uniform(0.0, 0.05, (ny, nx))
    n = rng.uniform(0.03, 0.05, (ny, nx))
    h0 = rng.uniform(0.2, 0.6, (ny, nx))
    l_in = ny if in_side in (WEST, EAST) else nx
    l_out = ny if out_side in (WEST, EAST) else nx
    ts = np.linspace(0, 100, 6)
    qs = np.array([5.0, 8.0, 12.0, 9.0, 6.0, 5.0])
    sc = _cast(Scenario("adj_sides", nx, ny, dx, z, n, h0, (in_side, l_in // 3, l_in // 3, S, ts, qs),
                        (out_side, 0, l_out, S), dt_max=0.5, dt_fixed=0.5), np.float64)
    gauges = rng.choice(nx * ny, NG, replace=False)
    truth, _, _, _ = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=np.zeros((N // OBS_EVERY, NG)),
                                    n=sc.n * 1.1)
    s_cpu, l_cpu, gn_cpu, gq_cpu = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=truth)
    print("CASE adjoint fp64 sides in=%d out=%d" % sides, flush=True)
    f, s, l, gn, gq = _gpu_adjoint(sc, "f64", gauges, truth)
    f.close()
    assert np.abs(s - s_cpu).max() <= 1e-11 * max(1.0, np.abs(s_cpu).max())
    assert abs(l / l_cpu - 1) <= 1e-8
    assert _rel_l2(gn, gn_cpu) <= 1e-8, _rel_l2(gn, gn_cpu)
    assert _rel_l2(gq, gq_cpu) <= 1e-8, _rel_l2(gq, gq_cpu)
    # the gradients reach the section's cells and the hydrograph
    assert np.abs(gq_cpu).max() > 0 and np.count_nonzero(gn_cpu) > nx * ny // 2


def test_fp32_gpu_adjoint_close_to_fp64():
    sc64 = _cast(_pin_scen(True), np.float64)
    sc32 = _cast(sc64, np.float32)
    sc64 = _cast(sc32, np.float64)     # both from the same float32 inputs
    rng = np.random.default_rng(6)
    gauges = rng.choice(sc64.nx * sc64.ny, NG, replace=False)
    truth, _, _, _ = oracle.adjoint(sc64, N, gauges, OBS_EVERY,
                                    obs=np.zeros((N // OBS_EVERY, NG)), n=sc64.n * 1.1)
    _, _, gn_cpu, gq_cpu = oracle.adjoint(sc64, N, gauges, OBS_EVERY, obs=truth)
    f, s, l, gn, gq = _gpu_adjoint(sc32, "f32", gauges, truth)
    f.close()
    assert _rel_l2(gn, gn_cpu) <= 1e-2
    cos = float(np.dot(gn.ravel(), gn_cpu.ravel()) /
                (np.linalg.norm(gn) * np.linalg.norm(gn_cpu)))
    assert cos >= 0.999
    assert _rel_l2(gq, gq_cpu) <= 1e-2


def test_fp64_gpu_adjoint_valley_against_cpu():
    """A 200 x 150 meandering valley, partly wet, 400 steps."""
    sc = _cast(_valley_scen(), np.float64)
    rng = np.random.default_rng(9)
    wet = np.nonzero(sc.h0.ravel() > 0.05)[0]
    gauges = rng.choice(wet, 40, replace=False)
    nsteps, obs_every = 400, 20
    truth, _, _, _ = oracle.adjoint(sc, nsteps, gauges, obs_every,
                                    obs=np.zeros((nsteps // obs_every, 40)), n=sc.n * 1.15)
    _, l_cpu, gn_cpu, gq_cpu = oracle.adjoint(sc, nsteps, gauges, obs_every, obs=truth)
    f, s, l, gn, gq = _gpu_adjoint(sc, "f64", gauges, truth, nsteps=nsteps, obs_every=obs_every)
    f.close()
    assert l_cpu > 0 and abs(l / l_cpu - 1) <= 1e-8
    assert _rel_l2(gn, gn_cpu) <= 1e-8
    assert _rel_l2(gq, gq_cpu) <= 1e-8


def test_fp64_gpu_adjoint_matches_finite_differences():
    sc = _cast(_pin_scen(True, seed=3), np.float64)
    rng = np.random.default_rng(4)
    gauges = rng.choice(sc.nx * sc.ny, NG, replace=False)
    truth, _, _, _ = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=np.zeros((N // OBS_EVERY, NG)),
                                    n=sc.n * 0.9)
    f, s, l, gn, gq = _gpu_adjoint(sc, "f64", gauges, truth)
    f.close()

    def loss(n=None, qs=None):
        sc2 = Scenario(sc.name, sc.nx, sc.ny, sc.dx, sc.z, sc.n if n is None else n, sc.h0,
                       sc.inflow if qs is None else sc.inflow[:5] + (qs,), sc.outflow,
                       dt_max=sc.dt_max, dt_fixed=sc.dt_fixed)
        g = fl.from_scenario(sc2, "f64")
        g.adj_setup(gauges, OBS_EVERY, truth)
        _, lv = g.adj_forward(N)
        g.close()
        return lv

    pairs = []
    for c in list(rng.choice(sc.nx * sc.ny, 5, replace=False)) + [3 * sc.nx, 6 * sc.nx]:
        j, i = divmod(int(c), sc.nx)
        eps = 1e-6 * sc.n[j, i]
        p, m = sc.n.copy(), sc.n.copy()
        p[j, i] += eps
        m[j, i] -= eps
        pairs.append((gn[j, i], (loss(n=p) - loss(n=m)) / (2 * eps)))
    qs0 = sc.inflow[5]
    for k in (1, 3):
        eps = 1e-6 * qs0[k]
        p, m = qs0.copy(), qs0.copy()
        p[k] += eps
        m[k] -= eps
        pairs.append((gq[k], (loss(qs=p) - loss(qs=m)) / (2 * eps)))
    scale = max(abs(fd) for _, fd in pairs)
    assert max(abs(a - fd) for a, fd in pairs) <= 1e-6 * scale


def test_forward_of_a_multi_step_context_gives_the_same_gradients():
    """A context committed with three steps per launch still makes the reverse
    mode's forward with single steps (the recompute relies on the step
    counter): the same series, loss and gradients, bit for bit."""
    sc = _cast(_valley_scen(nx=130, ny=90), np.float32)
    rng = np.random.default_rng(9)
    gauges = rng.choice(sc.nx * sc.ny, NG, replace=False)
    obs = rng.uniform(0.0, 0.5, (N // OBS_EVERY, NG))
    out = {}
    for k in (1, 3):
        print(f"CASE adjoint forward k={k}", flush=True)
        f = fl.from_scenario(sc, "f32", fusion=k)
        f.adj_setup(gauges, OBS_EVERY, obs.astype(f.dtype), 7)
        series, loss = f.adj_forward(N)
        gn, gq = f.adj_backward(None, len(sc.inflow[5]))
        h = f.get_depth()
        f.close()
        out[k] = (series, loss, gn, gq, h)
    for a, b in zip(out[3], out[1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_context_continues_after_the_backward_sweep():
    """After fl_adj_backward the context is back at the end of the forward run."""
    sc = _cast(_pin_scen(True), np.float32)
    rng = np.random.default_rng(2)
    gauges = rng.choice(sc.nx * sc.ny, NG, replace=False)
    f = fl.from_scenario(sc, "f32")
    f.adj_setup(gauges, OBS_EVERY, np.zeros((N // OBS_EVERY, NG), np.float32))
    f.adj_forward(N)
    f.adj_backward(None, 6)
    f.step(77)
    h = f.get_depth()
    r = f.get_report()
    f.close()
    g = fl.from_scenario(sc, "f32")
    g.step(N + 77)
    h2 = g.get_depth()
    r2 = g.get_report()
    g.close()
    assert np.array_equal(h, h2) and r.t == r2.t
    assert abs(r.v_out - r2.v_out) <= 1e-12 * max(1.0, r2.v_out)


def test_autograd_function_matches_direct_calls():
    import torch
    from paper_2204_10323_amd.autograd import gauge_series
    sc = _cast(_pin_scen(True), np.float64)
    rng = np.random.default_rng(5)
    gauges = rng.choice(sc.nx * sc.ny, NG, replace=False)
    truth, _, _, _ = oracle.adjoint(sc, N, gauges, OBS_EVERY, obs=np.zeros((N // OBS_EVERY, NG)),
                                    n=sc.n * 1.1)
    f, s, l, gn, gq = _gpu_adjoint(sc, "f64", gauges, truth)
    f.close()
    flood = fl.from_scenario(sc, "f64", commit=False)
    n_t = torch.tensor(sc.n, dtype=torch.float64, device="cuda", requires_grad=True)
    q_t = torch.tensor(sc.inflow[5], dtype=torch.float64, requires_grad=True)
    side, first, count, slope, ts, _ = sc.inflow
    series = gauge_series(flood, n_t, q_t, N, (side, first, count, slope, ts), gauges, OBS_EVERY)
    obs = torch.tensor(truth, device="cuda")
    loss = ((series - obs) ** 2).sum()
    loss.backward()
    assert abs(loss.item() / l - 1) <= 1e-12
    assert np.abs(n_t.grad.cpu().numpy() - gn).max() <= 1e-12 * np.abs(gn).max()
    assert np.abs(q_t.grad.numpy() - gq).max() <= 1e-12 * np.abs(gq).max()
    flood.close()


def test_adjoint_errors():
    sc = _cast(_pin_scen(True), np.float32)
    f = fl.from_scenario(sc, "f32", dt_fixed=0.0)
    with pytest.raises(fl.FloodError):
        f.adj_setup([1, 2], 10)               # needs a fixed dt
    f.close()
    g = fl.from_scenario(sc, "f32")
    with pytest.raises(fl.FloodError):
        g.adj_setup([sc.nx * sc.ny], 10)      # gauge outside the grid
    g.adj_setup([1, 2], 10)
    with pytest.raises(fl.FloodError) as ei:
        g.adj_backward(None, 6)               # no forward yet
    assert ei.value.status == fl.FL_ESTATE
    g.adj_forward(40)
    with pytest.raises(fl.FloodError):
        g.adj_backward(None, 6)               # no observations and no seeds
    g.step(1)
    with pytest.raises(fl.FloodError) as ei:
        g.adj_backward(np.ones((4, 2), np.float32), 6)   # stepped since the forward
    assert ei.value.status == fl.FL_ESTATE
    g.close()
