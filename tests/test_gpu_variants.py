"""GPU parity of the method variants (fl_set_variant) against the FP64 oracle.

Both sides implement the same two alternative readings: the vector-norm
friction term and the literal cell-area Manning boundaries.  Same gates as the
default method: every step of tiny random grids (FP64 1e-12, FP32 2e-5 of the
solution scale), the 256^2 valley after 2000 CFL steps (FP64 1e-10, FP32
1e-3 m, budgets), bitwise tiling invariance, and the combinations the library
refuses."""
import numpy as np
import pytest

import oracle
import paper_2204_10323_amd as fl
from gpu_util import max_abs, rel_err, run_gpu, run_oracle
from synth import config_d1, random_tiny

pytestmark = pytest.mark.gpu

VARIANTS = [("vector", "section"), ("face", "cell_area"), ("vector", "cell_area")]


def _orc(var):
    return dict(friction_vector=var[0] == "vector", boundary_cell_area=var[1] == "cell_area")


@pytest.mark.parametrize("var", VARIANTS)
@pytest.mark.parametrize("nx,ny", [(1, 1), (3, 2), (7, 9), (9, 7), (40, 23), (150, 70)])
def test_tiny_step_by_step(var, nx, ny):
    sc = random_tiny(nx, ny, 700 + nx * 10 + ny)
    for prec, tol in (("f64", 1e-12), ("f32", 2e-5)):
        print(f"CASE variant {var} tiny {nx}x{ny} {prec}", flush=True)
        f = fl.from_scenario(sc, prec, steps_per_graph=6, variant=var, cells_per_lane=1,
                             rows_per_item=4)
        o = oracle.Run(sc, **_orc(var))
        for step in range(12):
            f.step(1)
            o.step(1)
            h = f.get_depth()
            qx, qy = f.get_discharge()
            sh = max(np.abs(o.h).max(), 1e-3)
            sq = max(np.abs(o.qx).max(), np.abs(o.qy).max(), 1e-3)
            assert max_abs(h, o.h) <= tol * sh, (prec, step, max_abs(h, o.h))
            assert max_abs(qx, o.qx) <= tol * sq, (prec, step)
            assert max_abs(qy, o.qy) <= tol * sq, (prec, step)
        r = f.get_report()
        assert r.steps == o.clock.steps
        f.close()


@pytest.mark.parametrize("var", VARIANTS)
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_d1_valley_2000_steps(var, precision):
    sc = config_d1()
    print(f"CASE variant {var} d1 {precision}", flush=True)
    h, qx, qy, r = run_gpu(sc, sc.steps, precision, variant=var)
    o = run_oracle(sc, sc.steps, **_orc(var))
    assert r.steps == o.clock.steps == sc.steps
    if precision == "f64":
        assert rel_err(h, o.h) <= 1e-10
        assert rel_err(qx, o.qx) <= 1e-10
        assert rel_err(qy, o.qy) <= 1e-10
        assert r.budget_error() <= 1e-12
    else:
        assert max_abs(h, o.h) <= 1e-3
        assert r.budget_error() <= 1e-6
    assert abs(r.v_in / o.clock.v_in - 1) <= (1e-10 if precision == "f64" else 1e-5)
    # the variant is not the default method
    d = run_oracle(sc, sc.steps)
    assert max_abs(o.h, d.h) > 1e-3


@pytest.mark.parametrize("var", VARIANTS)
def test_tilings_bitwise(var):
    sc = random_tiny(301, 77, 31)
    ref = None
    for cpt, rows in [(1, 3), (2, 8), (4, 5), (1, 32)]:
        h, qx, qy, r = run_gpu(sc, 40, "f32", cells_per_lane=cpt, rows_per_item=rows, variant=var)
        if ref is None:
            ref = (h, qx, qy, r.t)
        else:
            assert np.array_equal(h, ref[0]) and np.array_equal(qx, ref[1])
            assert np.array_equal(qy, ref[2]) and r.t == ref[3]


def test_refused_combinations():
    sc = config_d1()
    L = fl.lib()
    for kw in (dict(fusion=2), dict(active_tiles=True)):
        f = fl.from_scenario(sc, "f32", variant=("vector", "section"), commit=False, **kw)
        assert L.fl_commit(f.ctx) == fl.FL_EINVAL
        f.close()
    f = fl.from_scenario(sc, "f32", variant=("face", "cell_area"))
    with pytest.raises(fl.FloodError):
        fl.Batch([f])
    g = fl.from_scenario(sc, "f64", variant=("vector", "section"), dt_fixed=0.5)
    with pytest.raises(fl.FloodError):
        g.adj_setup(np.array([100], np.int32), 10)
    with pytest.raises(ValueError):
        g.set_variant("diagonal", "section")
    assert L.fl_set_variant(g.ctx, 2, 0) == fl.FL_EINVAL
    f.step(10)                                   # the context itself still steps
    assert f.get_report().steps == 10
    f.close()
    g.close()
