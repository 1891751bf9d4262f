"""The batched ensemble (one persistent launch for many uneven grids).

Every member must end bitwise equal to the same scenario stepped alone (the
batch runs the same kernels on the same state), whatever the batch tiling;
the autotuner's trial steps must leave the state untouched; batch and single
steps can be interleaved; FP64 members agree with the oracle.
"""
import numpy as np
import pytest

import oracle
import paper_2204_10323_amd as fl
from gpu_util import max_abs, rel_err, run_gpu
from synth import EAST, NORTH, SOUTH, WEST, Scenario, Valley, manning_field, valley_dem64

pytestmark = pytest.mark.gpu


def _member(nx, ny, seed, side_in=WEST, side_out=EAST, peak=60.0):
    v = Valley(nx, ny, 5.0, 1e-3, 2.0, 30.0, 0.4, seed=seed, meander=True)
    z = valley_dem64(v).astype(np.float32)
    n = manning_field(v).astype(np.float32)
    L_in = ny if side_in in (WEST, EAST) else nx
    L_out = ny if side_out in (WEST, EAST) else nx
    c = max(1, L_in // 8)
    return Scenario(f"m{seed}", nx, ny, 5.0, z, n, np.zeros_like(z),
                    (side_in, (L_in - c) // 2, c, 1e-3, np.array([0.0, 200.0, 600.0]),
                     np.array([5.0, peak, 10.0])),
                    (side_out, 0, L_out, 1e-3), dt_max=0.5)


MEMBERS = [(37, 53, 1, WEST, EAST), (300, 256, 2, WEST, EAST), (600, 143, 3, SOUTH, NORTH),
           (999, 1000, 4, WEST, EAST), (64, 700, 5, NORTH, SOUTH), (257, 129, 6, EAST, WEST)]


def _scenarios():
    return [_member(nx, ny, seed, si, so) for nx, ny, seed, si, so in MEMBERS]


def _state(f):
    h = f.get_depth()
    qx, qy = f.get_discharge()
    return h, qx, qy, f.get_report()


@pytest.mark.parametrize("tiling", [(4, 16), (2, 5), (1, 64)])
def test_batch_members_equal_single_runs(tiling):
    scs = _scenarios()
    ref = [run_gpu(sc, 300, "f32") for sc in scs]
    members = [fl.from_scenario(sc, "f32") for sc in scs]
    b = fl.Batch(members)
    b.set_tiling(*tiling)
    print("CASE batch tiling", tiling, flush=True)
    b.run(300)
    for sc, f, (h0, qx0, qy0, r0) in zip(scs, members, ref):
        h, qx, qy, r = _state(f)
        assert np.array_equal(h, h0), sc.name
        assert np.array_equal(qx, qx0) and np.array_equal(qy, qy0), sc.name
        assert r.t == r0.t and r.steps == r0.steps == 300
        assert r.budget_error() <= 1e-6
        assert abs(r.v_out - r0.v_out) <= 1e-12 * max(1.0, r0.v_out)
    b.close()
    for f in members:
        f.close()


def test_autotune_leaves_state_unchanged_and_interleaving():
    scs = _scenarios()[:4]
    ref = [run_gpu(sc, 250, "f32") for sc in scs]
    members = [fl.from_scenario(sc, "f32") for sc in scs]
    for f in members:
        f.step(40)                 # some steps alone first (own tiling)
    b = fl.Batch(members)
    best, ms = b.autotune([(4, 8), (4, 32), (2, 16)], trial_steps=7)
    print("CASE autotune best", best, ms, flush=True)
    assert best in ((4, 8), (4, 32), (2, 16)) and ms > 0
    b.run(150)
    for f in members:
        f.step(60)                 # and alone again
    for sc, f, (h0, qx0, qy0, r0) in zip(scs, members, ref):
        h, qx, qy, r = _state(f)
        assert np.array_equal(h, h0), sc.name
        assert np.array_equal(qx, qx0) and np.array_equal(qy, qy0), sc.name
        assert r.t == r0.t and r.steps == 250
        assert abs(r.v_out - r0.v_out) <= 1e-12 * max(1.0, r0.v_out)
        assert abs(r.v_in - r0.v_in) <= 1e-12 * max(1.0, r0.v_in)
    b.close()
    for f in members:
        f.close()


def test_batch_fp64_members_match_oracle():
    scs = [_member(90, 61, 11), _member(130, 47, 12, SOUTH, NORTH), _member(40, 200, 13, NORTH, SOUTH)]
    members = [fl.from_scenario(sc, "f64") for sc in scs]
    b = fl.Batch(members)
    b.set_tiling(2, 8)
    b.run(400)
    for sc, f in zip(scs, members):
        h, qx, qy, r = _state(f)
        o = oracle.Run(sc)
        o.step(400)
        assert np.abs(o.h).max() > 0.05
        assert rel_err(h, o.h) <= 1e-10, sc.name
        assert rel_err(qx, o.qx) <= 1e-10 and rel_err(qy, o.qy) <= 1e-10, sc.name
        assert r.budget_error() <= 1e-12
    b.close()
    for f in members:
        f.close()


def test_batch_members_reach_t_end_independently():
    """A member whose t_end comes first stops there while the others go on."""
    scs = _scenarios()[:3]
    members = [fl.from_scenario(sc, "f32", t_end=(20.0 if k == 1 else float("inf")))
               for k, sc in enumerate(scs)]
    b = fl.Batch(members)
    b.run(100)
    r = [f.get_report() for f in members]
    assert r[1].t == 20.0 and r[1].done == 1 and r[1].steps < 100
    assert r[0].steps == 100 and r[2].steps == 100
    b.close()
    for f in members:
        f.close()


def test_batch_create_errors():
    sc = _scenarios()[0]
    f = fl.from_scenario(sc, "f32")
    g = fl.from_scenario(sc, "f64")
    with pytest.raises(fl.FloodError):
        fl.Batch([f, g])            # mixed precision
    with pytest.raises(fl.FloodError):
        fl.Batch([f, f])            # same context twice
    u = fl.from_scenario(sc, "f32", commit=False)
    with pytest.raises(fl.FloodError):
        fl.Batch([f, u])            # not committed
    b = fl.Batch([f])
    with pytest.raises(fl.FloodError):
        b.set_tiling(3, 8)
    f.set_params(dt_max=0.2)        # member changed after the batch was made
    with pytest.raises(fl.FloodError) as ei:
        b.run(1)
    assert ei.value.status == fl.FL_ESTATE
    b.close()
    with pytest.raises(ValueError):
        b.run(1)                    # the batch is closed
    f.commit()
    h = fl.from_scenario(sc, "f32")
    b2 = fl.Batch([f, h])
    h.close()                       # a member closed while the batch still borrows it
    with pytest.raises(ValueError):
        b2.run(1)
    b2.close()
    for x in (f, g, u):
        x.close()


# ---------------------------------------------------------------- two steps per entry
def _same2(a, b, what=""):
    """State, clock and inflow volume bit for bit; the outflow volume is summed
    over another work decomposition, so it agrees to FP64 rounding."""
    for x, y, nm in zip(a[:3], b[:3], ("h", "qx", "qy")):
        assert np.array_equal(x, y), f"{what}: {nm} differs"
    ra, rb = a[3], b[3]
    assert ra.steps == rb.steps and ra.t == rb.t and ra.last_dt == rb.last_dt, what
    assert ra.v_in == rb.v_in, what
    assert abs(ra.v_out - rb.v_out) <= 1e-13 * max(1.0, abs(rb.v_out)), what


def _basin():
    """A basin filled from the west whose CFL bound becomes active during the
    run: speculated second steps are redone, then launches make one step."""
    nx, ny = 96, 64
    z = np.fromfunction(lambda j, i: 0.002 * (nx - i) + 0.01 * np.sin(j / 5.0),
                        (ny, nx)).astype(np.float32)
    n = np.full((ny, nx), 0.03, np.float32)
    return Scenario("basin", nx, ny, 1.0, z, n, np.zeros_like(z),
                    (WEST, 20, 8, 1e-3, np.array([0.0, 50.0, 100.0]), np.array([400.0, 400.0, 0.0])),
                    (EAST, 0, ny, 1e-3), dt_max=1.0)


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("prec,tiling", [("f32", (2, 32)), ("f32", (1, 8)), ("f32", (2, 5)),
                                         ("f64", (1, 16)), ("f64", (2, 7))])
def test_multi_step_batch_members_equal_single_runs(prec, tiling, k):
    """Two or three steps per queue entry: each member ends as the same scenario
    stepped alone one step per launch (step counts that are no multiple of k, a
    member whose CFL bound becomes active, every side pair)."""
    scs = _scenarios() + [_basin()]
    chunks = [151, 150]
    ref = []
    for sc in scs:
        f = fl.from_scenario(sc, prec)
        for n in chunks:
            f.step(n)
        ref.append(_state(f))
        f.close()
    members = [fl.from_scenario(sc, prec, fusion=k) for sc in scs]
    b = fl.Batch(members)
    b.set_fusion(k, *tiling)
    print("CASE multi-step batch", k, prec, tiling, flush=True)
    for n in chunks:
        b.run(n)
    b.close()
    for sc, f, r0 in zip(scs, members, ref):
        _same2(_state(f), r0, sc.name)
        f.close()
    assert ref[-1][3].last_dt < 1.0   # the basin's bound became active


@pytest.mark.parametrize("k", [2, 3])
def test_multi_step_batch_autotune_and_interleaving(k):
    """The multi-step batch autotuner leaves states untouched; batched multi-step
    runs, one-step batch runs and the members' own steps interleave."""
    scs = _scenarios()
    ref = [run_gpu(sc, 260, "f32") for sc in scs]
    members = [fl.from_scenario(sc, "f32", fusion=k) for sc in scs]
    b = fl.Batch(members)
    b.set_fusion(k)
    best, _ = b.autotune([(2, 32), (1, 16), (2, 8)], 6)
    assert best in [(2, 32), (1, 16), (2, 8)]
    b.run(100)
    for f in members:
        f.step(21)
    b.set_fusion(1)
    b.run(39)
    b.set_fusion(k, *best)
    b.run(100)
    b.close()
    for sc, f, (h0, qx0, qy0, r0) in zip(scs, members, ref):
        h, qx, qy, r = _state(f)
        _same2((h, qx, qy, r), (h0, qx0, qy0, r0), sc.name)
        f.close()


def test_two_step_batch_refusals():
    scs = _scenarios()[:2]
    plain = [fl.from_scenario(sc, "f32") for sc in scs]
    b = fl.Batch(plain)
    with pytest.raises(fl.FloodError) as e:
        b.set_fusion(2)
    assert e.value.status == fl.FL_ESTATE
    with pytest.raises(fl.FloodError) as e:
        b.set_fusion(3)
    assert e.value.status == fl.FL_ESTATE
    with pytest.raises(fl.FloodError) as e:
        b.set_fusion(4)
    assert e.value.status == fl.FL_EINVAL
    b.close()
    act = [fl.from_scenario(sc, "f32", fusion=2, active_tiles=True) for sc in scs]
    b = fl.Batch(act)
    with pytest.raises(fl.FloodError) as e:
        b.set_fusion(2)
    assert e.value.status == fl.FL_EINVAL
    b.close()
    for f in plain + act:
        f.close()
