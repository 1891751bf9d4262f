"""Active-tile skipping (fl_set_active_tiles) against computing every work item.

A skipped item is one whose cells cannot change in the step, so both runs must
hold the same values after every call: depths, discharges (a zero may differ
in sign, which numpy's equality ignores), the clock and both volumes.  The
cases put dry ground between wet patches, start inflows late (the items
behind an inflow face are always computed), use work items down to one row,
and hand the state between skipping and non-skipping paths."""
import numpy as np
import pytest

import oracle
import paper_2204_10323_amd as fl
import synth
from gpu_util import max_abs
from synth import EAST, NORTH, SOUTH, WEST, Scenario, config_d1

pytestmark = pytest.mark.gpu


def _run(sc, prec, chunks, active, tiling=(0, 0), fusion=None, **params):
    """Step `sc` in calls of `chunks` steps (floats: fl_advance seconds);
    tiling is the single-step tiling, or with fusion = (2, cpt, rows) the
    two-step launches'."""
    f = fl.from_scenario(sc, prec, cells_per_lane=tiling[0], rows_per_item=tiling[1],
                         active_tiles=active, fusion=fusion, **params)
    out = []
    for n in chunks:
        if isinstance(n, float):
            f.advance(n)
        else:
            f.step(n)
        h = f.get_depth()
        qx, qy = f.get_discharge()
        r = f.get_report(check=False)
        out.append((h, qx, qy, r))
    f.close()
    return out


def _same(a, b, what="", other_decomposition=False):
    """Same values after every call.  The outflow volume is summed from
    per-work-item partials: against a run with another work decomposition
    (two steps per launch) it agrees to FP64 rounding."""
    for k, (x, y) in enumerate(zip(a, b)):
        for u, v, nm in zip(x[:3], y[:3], ("h", "qx", "qy")):
            assert np.array_equal(u, v), f"{what} call {k}: {nm} differs"
        ra, rb = x[3], y[3]
        assert (ra.steps, ra.t, ra.last_dt, ra.done, ra.nonfinite) == \
            (rb.steps, rb.t, rb.last_dt, rb.done, rb.nonfinite), f"{what} call {k}"
        assert ra.v_in == rb.v_in, f"{what} call {k}"
        if other_decomposition:
            assert abs(ra.v_out - rb.v_out) <= 1e-13 * max(1.0, abs(rb.v_out)), f"{what} call {k}"
        else:
            assert ra.v_out == rb.v_out, f"{what} call {k}"


def patchy(nx, ny, seed, t_on=1.0, sides=None):
    """Dry terrain with a few wet patches (still water with random discharges
    inside the patch), an inflow whose hydrograph is zero until t_on, an
    outflow on another side."""
    rng = np.random.default_rng(seed)
    jj, ii = np.mgrid[0:ny, 0:nx]
    z = synth._f32(rng.uniform(0.0, 0.3, (ny, nx)) + 0.004 * ii + 0.002 * jj)
    n = synth._f32(rng.uniform(0.02, 0.08, (ny, nx)))
    h = np.zeros((ny, nx))
    qx = np.zeros((ny, nx + 1))
    qy = np.zeros((ny + 1, nx))
    for _ in range(int(rng.integers(1, 4))):
        ci, cj = rng.integers(0, nx), rng.integers(0, ny)
        r = rng.uniform(2.0, 0.2 * max(nx, ny))
        disc = (ii - ci) ** 2 + (jj - cj) ** 2 <= r * r
        eta = z[disc].mean() + rng.uniform(0.1, 0.6)
        h[disc] = np.maximum(h[disc], eta - z[disc])
    wet = h > 0
    qx[:, 1:nx][wet[:, :-1] & wet[:, 1:]] = rng.normal(0, 0.2, (wet[:, :-1] & wet[:, 1:]).sum())
    qy[1:ny, :][wet[:-1, :] & wet[1:, :]] = rng.normal(0, 0.2, (wet[:-1, :] & wet[1:, :]).sum())
    side_in, side_out = sides if sides else [(WEST, EAST), (EAST, WEST), (SOUTH, NORTH),
                                             (NORTH, SOUTH)][int(rng.integers(0, 4))]
    L_in = ny if side_in in (WEST, EAST) else nx
    L_out = ny if side_out in (WEST, EAST) else nx
    c_in = int(rng.integers(1, max(2, L_in // 3)))
    f_in = int(rng.integers(0, L_in - c_in + 1))
    c_out = int(rng.integers(1, L_out + 1))
    f_out = int(rng.integers(0, L_out - c_out + 1))
    ts = np.array([0.0, t_on, t_on + 2.0])
    qs = np.array([0.0, 0.0, 3.0 * c_in])
    sc = Scenario(f"patchy_{nx}x{ny}_{seed}", nx, ny, 1.0, z, n, synth._f32(h),
                  (side_in, f_in, c_in, 1e-3, ts, qs), (side_out, f_out, c_out, 1e-3),
                  dt_max=0.05)
    sc.extra["qx0"] = synth._f32(qx)
    sc.extra["qy0"] = synth._f32(qy)
    return sc


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("prec,cpt", [("f32", 1), ("f32", 2), ("f32", 4), ("f64", 1), ("f64", 2)])
def test_valley256_2000_steps(prec, cpt, mode):
    """The 256^2 valley from a dry start: a flood that grows across the grid
    (mode 1: per-item skip test; mode 2: selected list)."""
    sc = config_d1()
    print(f"CASE valley256 active tiles {prec} cpt={cpt} mode {mode}", flush=True)
    chunks = [1, 50, 449, 1500]
    ref = _run(sc, prec, chunks, False, (cpt, 8))
    got = _run(sc, prec, chunks, mode, (cpt, 8))
    _same(got, ref, f"{prec} cpt={cpt}")


def test_valley256_matches_oracle():
    """The skipping run against the FP64 oracle at the FP32 gate."""
    sc = config_d1()
    got = _run(sc, "f32", [2000], True, (2, 8))[-1]
    o = oracle.Run(sc)
    o.step(2000)
    assert max_abs(got[0], o.h) <= 1e-3
    assert got[3].budget_error() <= 1e-6


@pytest.mark.parametrize("seed", range(10))
def test_patchy_grids_small_items(seed):
    """Wet patches on dry ground, a late inflow, work items of 1 to 5 rows and
    1, 2 or 4 cells per lane (several strips), CFL clock, FP32 and FP64."""
    rng = np.random.default_rng(1000 + seed)
    nx, ny = int(rng.integers(20, 300)), int(rng.integers(10, 120))
    sc = patchy(nx, ny, 2000 + seed)
    cpt = [1, 2, 4][seed % 3]
    rows = [1, 2, 3, 5][seed % 4]
    chunks = [1, 1, 7, 30, 3, 60]
    for prec in ("f32", "f64"):
        if prec == "f64" and cpt == 4:
            continue
        ref = _run(sc, prec, chunks, False, (cpt, rows))
        for mode in (1, 2):
            print(f"CASE patchy {nx}x{ny} seed {seed} {prec} cpt={cpt} rows={rows} mode {mode}",
                  flush=True)
            got = _run(sc, prec, chunks, mode, (cpt, rows))
            _same(got, ref, f"patchy {nx}x{ny} {prec} mode {mode}")


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("side", [WEST, EAST, SOUTH, NORTH])
def test_late_inflow_every_side(side, mode):
    """A dry grid whose inflow starts at t = 1 s: while it is zero only the
    items behind the inflow faces are computed; then the flood spreads."""
    nx, ny, cpt, rows = 200, 90, 1, 4
    sc = patchy(nx, ny, 77, t_on=1.0, sides=(side, [EAST, WEST, NORTH, SOUTH][side]))
    sc.h0[:] = 0
    sc.extra["qx0"][:] = 0
    sc.extra["qy0"][:] = 0
    f = fl.from_scenario(sc, "f32", cells_per_lane=cpt, rows_per_item=rows, active_tiles=mode)
    f.step(10)                                  # 0.5 s: the inflow is still zero
    nxt, tot = f.active_items()
    wo = 64 * cpt - 4
    ns, nc = -(-nx // wo), -(-ny // rows)
    assert tot == ns * nc
    s_in, first, count = sc.inflow[0], sc.inflow[1], sc.inflow[2]
    if s_in in (WEST, EAST):
        pinned = len({j // rows for j in range(first, first + count)})
    else:
        pinned = len({i // wo for i in range(first, first + count)})
    assert nxt == pinned, (nxt, pinned)
    assert not f.get_depth().any()
    f.close()
    chunks = [10, 30, 100]
    ref = _run(sc, "f32", chunks, False, (cpt, rows))
    got = _run(sc, "f32", chunks, mode, (cpt, rows))
    _same(got, ref, f"side {side}")
    assert got[-1][0].max() > 0.01


@pytest.mark.parametrize("mode", [1, 2])
def test_dry_closed_grid_computes_nothing(mode):
    nx, ny = 300, 64
    z = synth._f32(np.random.default_rng(3).uniform(0, 1, (ny, nx)))
    n = np.full((ny, nx), 0.03, np.float32)
    sc = Scenario("dry", nx, ny, 1.0, z, n, np.zeros_like(z), None, None, dt_max=0.05)
    f = fl.from_scenario(sc, "f32", cells_per_lane=2, rows_per_item=8, active_tiles=mode)
    nxt, tot = f.active_items()
    assert nxt == tot                           # before any step: everything
    f.step(1)
    assert f.active_items()[0] == tot           # the item's own flag two steps back is still 1
    f.step(1)
    assert f.active_items()[0] == 0
    f.step(100)
    assert f.active_items()[0] == 0
    r = f.get_report()
    assert r.steps == 102 and not f.get_depth().any()
    f.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_state_handed_between_paths(mode):
    """Skipping steps, then a batch run, frozen tiling trials (which may switch
    the skip mode), fl_advance and skipping steps again: the flags are
    refreshed whenever another path moved the state."""
    sc = patchy(180, 70, 5)
    ref = _run(sc, "f32", [5, 20, 7, 3.0, 40], False, (1, 4))
    f = fl.from_scenario(sc, "f32", cells_per_lane=1, rows_per_item=4, active_tiles=mode)
    f.step(5)
    b = fl.Batch([f])
    b.run(20)
    b.close()
    f.autotune([(1, 4), (2, 3), (1, 2)], 3)      # frozen trial steps, then a new tiling
    f.step(7)
    f.advance(3.0)
    f.step(40)
    h = f.get_depth()
    qx, qy = f.get_discharge()
    r = f.get_report(check=False)
    f.close()
    _same([(h, qx, qy, r)], [ref[-1]], "handed")


def test_reverse_mode_forward_with_active_tiles():
    """The forward of reverse mode steps with skipping; its series, loss and
    gradients equal those of a context without."""
    sc = patchy(120, 60, 9)
    sc.dt_fixed = 0.05
    rng = np.random.default_rng(4)
    gauges = rng.choice(sc.nx * sc.ny, 20, replace=False).astype(np.int32)
    res = []
    for active in (False, True):
        f = fl.from_scenario(sc, "f64", active_tiles=active)
        f.adj_setup(gauges, 10, np.zeros((6, 20)), 0)
        series, loss = f.adj_forward(60)
        gn, gq = f.adj_backward(nsamples=3)
        f.step(5)                                # stepping continues after the sweep
        res.append((series, loss, gn, gq, f.get_depth()))
        f.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


@pytest.mark.parametrize("k", [2, 3])
def test_k_steps_per_launch_need_k_row_items(k):
    sc = config_d1()
    f = fl.from_scenario(sc, "f32", fusion=(k, 2, k - 1), active_tiles=True, commit=False)
    assert fl.lib().fl_commit(f.ctx) == fl.FL_EINVAL
    f.set_fusion(k, 2, k)
    f.commit()
    f.step(6)
    f.close()


# ------------------------------------------- with two or three steps per launch
@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("prec,cpt", [("f32", 1), ("f32", 2), ("f32", 4), ("f64", 1), ("f64", 2)])
def test_multi_step_valley256_2000_steps(prec, cpt, k):
    """Two or three steps per launch with skipping against one step per launch
    that computes everything (the two paths give the same bits)."""
    if cpt == 4 and k == 3:
        pytest.skip("4 cells per lane run two steps per launch at most")
    sc = config_d1()
    print(f"CASE {k}-step valley256 active tiles {prec} cpt={cpt}", flush=True)
    chunks = [1, 50, 449, 1500]
    ref = _run(sc, prec, chunks, False, (cpt if cpt < 4 or prec == "f32" else 2, 8))
    got = _run(sc, prec, chunks, True, fusion=(k, cpt, 8))
    _same(got, ref, f"{prec} cpt={cpt}", other_decomposition=True)


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("seed", range(8))
def test_multi_step_patchy_grids(seed, k):
    rng = np.random.default_rng(3000 + seed)
    nx, ny = int(rng.integers(20, 300)), int(rng.integers(10, 120))
    sc = patchy(nx, ny, 4000 + seed)
    cpt = [1, 2][seed % 2]
    rows = max(k, [2, 3, 5, 8][seed % 4])
    chunks = [1, 2, 7, 30, 3, 61]
    for prec in ("f32", "f64"):
        print(f"CASE {k}-step patchy {nx}x{ny} seed {seed} {prec} cpt={cpt} rows={rows}", flush=True)
        ref = _run(sc, prec, chunks, False, (1, 4))
        got = _run(sc, prec, chunks, True, fusion=(k, cpt, rows))
        _same(got, ref, f"two-step patchy {nx}x{ny} {prec}", other_decomposition=True)


@pytest.mark.parametrize("k", [2, 3])
def test_multi_step_cfl_becomes_active_with_skipping(k):
    """A basin filled from one side: the speculated dt of the second step
    turns wrong, launches redo, then make one step each; meanwhile most of the
    basin is dry and skipped."""
    nx, ny = 300, 64
    z = synth._f32(np.fromfunction(lambda j, i: 0.002 * (nx - i) + 0.01 * np.sin(j / 5.0),
                                   (ny, nx)))
    n = np.full((ny, nx), 0.03, np.float32)
    ts, qs = np.array([0.0, 50.0, 100.0]), np.array([400.0, 400.0, 0.0])
    sc = Scenario("basin", nx, ny, 1.0, z, n, np.zeros_like(z),
                  (WEST, 20, 8, 1e-3, ts, qs), (EAST, 0, ny, 1e-3), dt_max=1.0)
    chunks = [150, 151, 40]
    ref = _run(sc, "f32", chunks, False, (1, 4))
    got = _run(sc, "f32", chunks, True, fusion=(k, 1, 4))
    _same(got, ref, "basin", other_decomposition=True)
    assert ref[-1][3].last_dt < sc.dt_max


@pytest.mark.parametrize("k", [2, 3])
def test_multi_step_and_single_step_skipping_interleaved(k):
    """fl_step(1) (single-step launch), fl_advance (single-step launches) and
    multi-step runs, all skipping, hand the state to each other."""
    sc = patchy(200, 90, 12)
    seq = [1, 9, 2.0, 40, 1, 1, 33, 3.5, 20]
    ref = _run(sc, "f32", seq, False, (1, 4))
    got = _run(sc, "f32", seq, True, (2, 8), fusion=(k, 2, 8))
    _same(got, ref, "interleaved", other_decomposition=True)


def test_workspace_holds_the_flags():
    import torch
    sc = config_d1()
    f = fl.from_scenario(sc, "f32", active_tiles=True, commit=False)
    need = f.workspace_bytes(active_tiles=True)
    assert need > f.workspace_bytes()
    small = torch.empty(f.workspace_bytes(), dtype=torch.uint8, device="cuda")
    f.bind_workspace(small)
    assert fl.lib().fl_commit(f.ctx) == fl.FL_EINVAL
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    f.bind_workspace(buf)
    f.commit()
    f.step(300)
    h = f.get_depth()
    f.close()
    ref = _run(sc, "f32", [300], False)[-1][0]
    assert np.array_equal(h, ref)


@pytest.mark.parametrize("k", [2, 3])
def test_multi_step_short_calls_keep_their_flags(k):
    """Many short multi-step calls in a row: the flags carry over from one call
    to the next (nothing else moved the state), and the state stays that of
    computing everything."""
    sc = patchy(240, 100, 21)
    chunks = [4] * 25 + [3, 6, 2]
    ref = _run(sc, "f32", chunks, False, (1, 4))
    got = _run(sc, "f32", chunks, True, fusion=(k, 2, 8))
    _same(got, ref, "short calls", other_decomposition=True)


@pytest.mark.parametrize("k", [2, 3])
def test_multi_step_dry_closed_grid_computes_nothing(k):
    nx, ny = 300, 64
    z = synth._f32(np.random.default_rng(3).uniform(0, 1, (ny, nx)))
    n = np.full((ny, nx), 0.03, np.float32)
    sc = Scenario("dry", nx, ny, 1.0, z, n, np.zeros_like(z), None, None, dt_max=0.05)
    f = fl.from_scenario(sc, "f32", fusion=(k, 2, 8), active_tiles=True)
    f.step(10)
    nxt, tot = f.active_items()
    w = 128 - 4 * k
    assert tot == -(-(nx - (2 * k - 2)) // w) * (ny // 8) and nxt == 0, (nxt, tot)
    f.step(10)
    assert f.active_items()[0] == 0
    assert f.get_report().steps == 20 and not f.get_depth().any()
    f.close()


@pytest.mark.parametrize("k", [2, 3])
def test_autotune_fusion_with_active_tiles_keeps_the_bits(k):
    sc = patchy(200, 90, 33)
    ref = _run(sc, "f32", [60], False, (2, 8))
    f = fl.from_scenario(sc, "f32", fusion=(k, 2, 8), cells_per_lane=2, rows_per_item=8,
                         active_tiles=True)
    f.step(20)
    spl, ms = f.autotune_fusion(10)
    assert spl in (1, k) and ms > 0
    f.step(40)
    h = f.get_depth()
    qx, qy = f.get_discharge()
    r = f.get_report(check=False)
    f.close()
    _same([(h, qx, qy, r)], [ref[-1]], "autotune_fusion", other_decomposition=True)


def _snap(f):
    h = f.get_depth()
    qx, qy = f.get_discharge()
    return h, qx, qy, f.get_report(check=False)


@pytest.mark.parametrize("own,batch", [((1, 4), (2, 8)), ((2, 8), (2, 8))])
def test_batch_members_with_active_tiles(own, batch):
    """Members with and without active tiles stepped by one batch, before and
    after steps of their own: the values of computing every item.  With the
    same tiling in the batch and alone the flags carry over."""
    scs = [patchy(180, 70, 41), patchy(260, 90, 42), patchy(90, 150, 43)]
    chunks = [5, 30, 20]
    refs = [_run(sc, "f32", chunks, False, (1, 4)) for sc in scs]
    fs = [fl.from_scenario(sc, "f32", cells_per_lane=own[0], rows_per_item=own[1],
                           active_tiles=(k != 1)) for k, sc in enumerate(scs)]
    got = [[] for _ in scs]
    for k, f in enumerate(fs):
        f.step(chunks[0])
        got[k].append(_snap(f))
    b = fl.Batch(fs)
    b.set_tiling(*batch)
    b.run(chunks[1])
    b.close()
    for k, f in enumerate(fs):
        got[k].append(_snap(f))
        f.step(chunks[2])
        got[k].append(_snap(f))
        f.close()
        _same(got[k], refs[k], f"member {k}", other_decomposition=True)


def test_batch_autotune_with_active_members_keeps_the_bits():
    scs = [patchy(200, 80, 51), patchy(150, 120, 52)]
    refs = [_run(sc, "f32", [60], False, (1, 4)) for sc in scs]
    fs = [fl.from_scenario(sc, "f32", active_tiles=True) for sc in scs]
    b = fl.Batch(fs)
    b.run(10)
    b.autotune([(2, 8), (1, 4), (4, 16)], 5)
    b.run(50)
    b.close()
    for f, ref in zip(fs, refs):
        _same([_snap(f)], [ref[-1]], "batch autotune", other_decomposition=True)
        f.close()
