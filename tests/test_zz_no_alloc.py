"""fl_batch_run_noalloc (the batch run for callers that cannot allocate; its
scratch is the library's static device array) against fl_batch_run on the same
members: the same depths, discharges, clocks and budgets, bit for bit (the bar
of the batch path), on two calls in a row, the second with a smaller batch of
smaller grids; and the member limit of the static array."""
import numpy as np
import pytest

import paper_2204_10323_amd as fl
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


FIRST = [(37, 53, 1, WEST, EAST), (300, 256, 2, WEST, EAST), (600, 143, 3, SOUTH, NORTH),
         (999, 1000, 4, WEST, EAST), (64, 700, 5, NORTH, SOUTH), (257, 129, 6, EAST, WEST)]
SECOND = [(41, 29, 7, WEST, EAST), (130, 90, 8, SOUTH, NORTH), (19, 77, 9, EAST, WEST)]


def _state(f):
    h = f.get_depth()
    qx, qy = f.get_discharge()
    r = f.get_report()
    return h, qx, qy, (r.t, r.steps, r.v_in, r.v_out, r.v_now)


def _compare(specs, steps, tiling):
    scs = [_member(*m) for m in specs]
    ref = [fl.from_scenario(sc, "f32") for sc in scs]
    new = [fl.from_scenario(sc, "f32") for sc in scs]
    b_ref, b_new = fl.Batch(ref), fl.Batch(new)
    b_ref.set_tiling(*tiling)
    b_new.set_tiling(*tiling)
    b_ref.run(steps)
    b_new.run_noalloc(steps)
    b_ref.close()
    b_new.close()
    for sc, f, g in zip(scs, ref, new):
        a, b = _state(f), _state(g)
        assert np.array_equal(a[0], b[0]), sc.name
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]), sc.name
        assert a[3] == b[3], sc.name
        assert a[3][1] == steps
        f.close()
        g.close()


def test_noalloc_batch_matches_batch_run_twice_second_smaller():
    print("CASE noalloc batch: 6 members, 300 steps", flush=True)
    _compare(FIRST, 300, (4, 16))
    print("CASE noalloc batch: 3 smaller members, 120 steps", flush=True)
    _compare(SECOND, 120, (2, 8))


def test_noalloc_batch_refuses_more_members_than_the_scratch_holds():
    print("CASE noalloc batch: member limit", flush=True)
    rng = np.random.default_rng(3)
    z = rng.uniform(0, 1, (8, 8)).astype(np.float32)
    n = np.full((8, 8), 0.03, np.float32)
    ctxs = []
    for _ in range(fl.FL_NOALLOC_MAX_MEMBERS + 1):
        f = fl.Flood(8, 8, 1.0, "f32")
        f.set_dem(z)
        f.set_manning(n)
        f.commit()
        ctxs.append(f)
    b = fl.Batch(ctxs)
    with pytest.raises(fl.FloodError) as e:
        b.run_noalloc(1)
    assert e.value.status == fl.FL_EINVAL and "at most" in str(e.value)
    b.close()
    # the same members within the limit run
    b = fl.Batch(ctxs[:fl.FL_NOALLOC_MAX_MEMBERS])
    b.run_noalloc(2)
    b.close()
    for f in ctxs:
        f.close()
