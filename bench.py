#!/usr/bin/env python3
"""Benchmark of the flood step on one MI355X.

Default workload: the 16384 x 16384 synthetic valley at dx = 1 m (268 M cells),
pre-wetted to the 30th percentile of the bed (every face carries water and runs
the face update of eq. 3), CFL time step, FP32 state.  One "step" is one full
time step of the method (device clock, boundary conditions, eq. 3 face update,
donor scaling, eq. 4 depth update, deepest-cell reduction), two per launch,
captured in HIP graphs.  Prints one JSON line: Gcell-updates/s, the HBM
roofline of the step kernel, and the FP64 CPU oracle timed on a bounded sample
of the same workload; `extras` holds the dry start of the same grid, active
tiles, the ensemble, the adjoint, the discharge sweep, the method variants and
the measured copy ceilings.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload valley16384]
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, AMD published
BYTES_PER_CELL = {"f32": 32, "f64": 64}   # read h z n qx qy, write h qx qy
CSRC = os.path.join(ROOT, "paper_2204_10323_amd", "csrc")
# the sources that make the step kernels' code
KERNEL_SRCS = ["flood_internal.h", "flood_device.h", "flood_march.h", "flood_kernels.hip",
               "flood_fused.hip"]
# committed PMC summaries of the dominant kernel, by steps per launch
PMC_SUMMARY = {1: os.path.join(ROOT, "profiles", "k_step_valley16384_pmc.md"),
               2: os.path.join(ROOT, "profiles", "k_fused2_valley16384_prewetted_pmc.md"),
               3: os.path.join(ROOT, "profiles", "k_fused3_valley16384_prewetted_pmc.md")}
PROBE_LIB = os.path.join(ROOT, "bench_probe.so")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SRCS:
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


# SQ counters of the dominant kernel (VALU busy): what bounds it
SQ_SUMMARY = {3: os.path.join(ROOT, "profiles", "k_fused3_valley16384_prewetted_sq_counters.md")}


def measured_valu_busy(fusion: int):
    """VALU busy of the dominant kernel from the committed SQ-counter summary,
    if it was taken on the current kernel sources; else None."""
    try:
        txt = open(SQ_SUMMARY[fusion]).read()
    except (OSError, KeyError):
        return None
    m = re.search(r"```json\s*(\{.*?\})\s*```", txt, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    return d.get("valu_busy") if d.get("kernel_sha256_16") == kernel_hash() else None


def measured_traffic(cells: int, fusion: int, workload: str):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary, if it was taken on the current kernel sources and this workload;
    else None."""
    try:
        txt = open(PMC_SUMMARY[fusion]).read()
    except (OSError, KeyError):
        return None
    m = re.search(r"```json\s*(\{.*?\})\s*```", txt, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if (d.get("kernel_sha256_16") != kernel_hash() or d.get("cells") != cells or
            d.get("workload") != workload):
        return None
    return d.get("hbm_bytes_per_launch")


def probe_stream(nbytes: int, reps: int, variant: int) -> float:
    """GB/s (read + write) of a plain stream (bench_probe.so): 1 kernel copy,
    4 read only, 5 write only, 7 the HIP runtime's device-to-device copy."""
    import ctypes as C
    L = C.CDLL(PROBE_LIB)
    L.probe_stream.restype = C.c_int
    L.probe_stream.argtypes = [C.c_int, C.c_size_t, C.c_int, C.c_int, C.POINTER(C.c_double)]
    g = C.c_double()
    st = L.probe_stream(0, int(nbytes), int(reps), int(variant), C.byref(g))
    if st != 0:
        raise RuntimeError(f"probe_stream variant {variant} failed with status {st}")
    return g.value


WORKLOAD_NAMES = {"valley16384": "valley_16384x16384_dx1m_dry_start",
                  "valley16384_wet": "valley_16384x16384_dx1m_prewetted"}


def build_workload(name: str):
    import synth
    if name == "valley16384":
        return synth.config_d3(16384, wet=False), WORKLOAD_NAMES[name]
    if name == "valley16384_wet":
        return synth.config_d3(16384, wet=True), WORKLOAD_NAMES[name]
    if name == "valley2048":
        return synth.config_d2(), "valley_2048x2048_dx5m_dry_start"
    if name == "valley256":
        return synth.config_d1(), "valley_256x256_dx10m_dry_start"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(sc, budget_s: float = 20.0):
    """The FP64 oracle on the same workload, from the same initial state, for as
    many whole steps as fit in about `budget_s` seconds (at least one)."""
    import numpy as np
    import oracle
    o = oracle.Run(sc, nthreads=0)
    cores = oracle.threads_used(0)
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    nmore = max(0, min(int(budget_s / max(one, 1e-6)) - 1, 50))
    if nmore:
        o.step(nmore)
    el = time.perf_counter() - t0
    steps = 1 + nmore
    val = sc.nx * sc.ny * steps / el / 1e9
    del o
    return {"value": round(val, 5), "unit": "Gcell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, first {steps} step(s) of the same {sc.nx}x{sc.ny} workload "
                      f"from the same initial state, {el:.1f} s wall on {cores} host threads"}


def cpu_single_thread(sc):
    """The FP64 oracle on one host thread: the first step of the same workload;
    with the host's CPU model."""
    import oracle
    o = oracle.Run(sc, nthreads=1)
    t0 = time.perf_counter()
    o.step(1)
    el = time.perf_counter() - t0
    del o
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"gcell_s": round(sc.nx * sc.ny / el / 1e9, 5), "threads": oracle.threads_used(1),
            "sample": f"FP64 oracle, first step of the {sc.nx}x{sc.ny} workload, {el:.1f} s wall",
            "host_cpu": model, "host_logical_cpus": os.cpu_count()}


# (cells per lane, rows per work item) tried by the autotuner on small grids
SMALL_GRID_TILINGS = [(1, 4), (1, 8), (2, 4), (2, 8), (4, 8), (4, 16), (4, 32)]
# ... and by the batch autotuner on the 64-member ensemble, one step per queue
# entry and two (the two-step tiling)
BATCH_TILINGS = [(4, 8), (4, 16), (4, 32), (4, 64), (2, 16), (2, 32)]
BATCH2_TILINGS = [(2, 32), (2, 64), (2, 96), (2, 128), (1, 64)]


def progress(msg: str):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_ensemble(fl, torch, steps: int, members: int = 64, trial_steps: int = 20):
    """64 valleys of uneven size (sides log-uniform in [256, 2048]) for `steps`
    steps: one persistent batch launch vs the same members one after another."""
    import synth
    sizes = synth.ensemble_sizes(members)
    scs = [synth.config_d4_member(s, side, steps) for s, side in enumerate(sizes)]
    cells = sum(sc.nx * sc.ny for sc in scs)
    stream = torch.cuda.current_stream().cuda_stream
    ctxs = [fl.from_scenario(sc, "f32", stream=stream) for sc in scs]
    # one after another: each member's own step kernel (autotuned) with graph replays
    seq_ms = 0.0
    for f in ctxs:
        f.autotune(SMALL_GRID_TILINGS, 10)
        f.step(3)
        seq_ms += f.time_steps(steps)
    progress("ensemble: members one after another, one step per launch, done")
    # one after another with two steps per launch
    seq2_ms = 0.0
    for sc in scs:
        g = fl.from_scenario(sc, "f32", stream=stream, fusion=2)
        g.step(3)
        seq2_ms += g.time_steps(steps)
        g.close()
    progress("ensemble: members one after another, two steps per launch, done")
    # one after another with three steps per launch
    seq3_ms = 0.0
    for sc in scs:
        g = fl.from_scenario(sc, "f32", stream=stream, fusion=3)
        g.step(3)
        seq3_ms += g.time_steps(steps)
        g.close()
    progress("ensemble: members one after another, three steps per launch, done")
    seq_best = min(seq_ms, seq2_ms, seq3_ms)
    b = fl.Batch(ctxs)
    cands = BATCH_TILINGS
    best, _ = b.autotune(cands, trial_steps)
    batch_ms = b.time(steps)
    rep = [f.get_report() for f in ctxs]
    b.close()
    for f in ctxs:
        f.close()
    def multi_step_batch(k):
        """The same members from the same start, k steps per queue entry."""
        ctxk = [fl.from_scenario(sc, "f32", stream=stream, fusion=k) for sc in scs]
        bk = fl.Batch(ctxk)
        bk.set_fusion(k)
        bestk, _ = bk.autotune(BATCH2_TILINGS, trial_steps)
        ms = bk.time(steps)
        repk = [f.get_report() for f in ctxk]
        bk.close()
        for f in ctxk:
            f.close()
        return bestk, ms, repk

    progress("ensemble: batch done; two steps per queue entry")
    best2, batch2_ms, rep2 = multi_step_batch(2)
    progress("ensemble: three steps per queue entry")
    best3, batch3_ms, rep3 = multi_step_batch(3)
    progress("ensemble: with active tiles")
    # the same members from the same start with active tiles (tilings autotuned
    # on skipping trial steps): batched, and one after another
    actx = [fl.from_scenario(sc, "f32", stream=stream, active_tiles=True) for sc in scs]
    ba = fl.Batch(actx)
    best_a, _ = ba.autotune(cands + [(2, 8), (1, 8)], trial_steps)
    batch_act_ms = ba.time(steps)
    rep_a = [f.get_report() for f in actx]
    ba.close()
    for f in actx:
        f.close()
    seq_act_ms = 0.0
    for sc in scs:
        g = fl.from_scenario(sc, "f32", stream=stream, active_tiles=True)
        g.autotune(SMALL_GRID_TILINGS, 10)
        g.step(3)
        seq_act_ms += g.time_steps(steps)
        g.close()
    return {"members": members, "sides": [min(sizes), max(sizes)], "cells": cells, "steps": steps,
            "active_tiles": {"batch_tiling_autotuned": list(best_a),
                             "batch_gcell_s_grid_equivalent": round(cells * steps / (batch_act_ms / 1e3) / 1e9, 3),
                             "sequential_gcell_s_grid_equivalent": round(cells * steps / (seq_act_ms / 1e3) / 1e9, 3),
                             "batch_vs_sequential": round(seq_act_ms / batch_act_ms, 3),
                             "batch_vs_full_batch": round(batch_ms / batch_act_ms, 3),
                             "max_budget_error": max(r.budget_error() for r in rep_a)},
            "tiling_autotuned": list(best),
            "batch_gcell_s": round(cells * steps / (batch_ms / 1e3) / 1e9, 3),
            "two_step_batch": {"tiling_autotuned": list(best2),
                               "gcell_s": round(cells * steps / (batch2_ms / 1e3) / 1e9, 3),
                               "vs_one_step_batch": round(batch_ms / batch2_ms, 3),
                               "vs_sequential": round(seq_ms / batch2_ms, 3),
                               "hbm_frac_one_pass_per_two_steps": round(
                                   16 * cells * steps / (batch2_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                               "max_budget_error": max(r.budget_error() for r in rep2)},
            "three_step_batch": {"tiling_autotuned": list(best3),
                                 "gcell_s": round(cells * steps / (batch3_ms / 1e3) / 1e9, 3),
                                 "vs_one_step_batch": round(batch_ms / batch3_ms, 3),
                                 "vs_two_step_batch": round(batch2_ms / batch3_ms, 3),
                                 "vs_sequential": round(seq_ms / batch3_ms, 3),
                                 "hbm_frac_one_pass_per_three_steps": round(
                                     32 / 3 * cells * steps / (batch3_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "max_budget_error": max(r.budget_error() for r in rep3)},
            "sequential_gcell_s": round(cells * steps / (seq_ms / 1e3) / 1e9, 3),
            "batch_vs_sequential": round(seq_ms / batch_ms, 3),
            "sequential_two_step_gcell_s": round(cells * steps / (seq2_ms / 1e3) / 1e9, 3),
            "sequential_three_step_gcell_s": round(cells * steps / (seq3_ms / 1e3) / 1e9, 3),
            "best_sequential_gcell_s": round(cells * steps / (seq_best / 1e3) / 1e9, 3),
            "batch_vs_best_sequential": round(seq_best / batch_ms, 3),
            "best_batch_gcell_s": round(cells * steps / (min(batch_ms, batch2_ms, batch3_ms) / 1e3) / 1e9, 3),
            "best_batch_vs_best_sequential": round(seq_best / min(batch_ms, batch2_ms, batch3_ms), 3),
            "batch_hbm_frac": round(32 * cells * steps / (batch_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "max_budget_error": max(r.budget_error() for r in rep)}


def run_adjoint(fl, torch, steps: int = 5000, nx: int = 1024, ngauges: int = 500,
                obs_every: int = 50):
    """1024^2 valley, fixed dt 0.25 s: gradient of the gauge misfit against a run
    with perturbed roughness, forward + checkpointed backward, vs the plain step."""
    import numpy as np
    import synth
    sc = synth.config_d5(nx, steps)
    stream = torch.cuda.current_stream().cuda_stream
    cells = sc.nx * sc.ny
    # the plain step on the same grid
    f = fl.from_scenario(sc, "f32", stream=stream)
    best, _ = f.autotune(SMALL_GRID_TILINGS, 10)
    f.step(6)
    plain_ms = f.time_steps(steps)
    f.close()
    f = fl.from_scenario(sc, "f32", stream=stream, fusion=2)
    f.step(6)
    plain2_ms = f.time_steps(steps)
    f.close()
    f = fl.from_scenario(sc, "f32", stream=stream, fusion=3)
    f.step(6)
    plain3_ms = f.time_steps(steps)
    f.close()
    # truth run with n_true, gauges among its wet cells at the last step
    truth = synth.Scenario(sc.name, sc.nx, sc.ny, sc.dx, sc.z, sc.extra["n_true"], sc.h0,
                           sc.inflow, sc.outflow, dt_max=sc.dt_max, dt_fixed=sc.dt_fixed)
    t = fl.from_scenario(truth, "f32", stream=stream)
    t.step(steps)
    h_end = t.get_depth()
    t.close()
    rng = np.random.default_rng(55)
    gauges = rng.choice(np.nonzero(h_end.ravel() > 0.05)[0], ngauges, replace=False)
    t = fl.from_scenario(truth, "f32", stream=stream)
    t.adj_setup(gauges, obs_every)
    obs, _ = t.adj_forward(steps)
    t.close()
    m = fl.from_scenario(sc, "f32", stream=stream)
    m.autotune(SMALL_GRID_TILINGS, 10)
    m.adj_setup(gauges, obs_every, obs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, loss = m.adj_forward(steps)
    t1 = time.perf_counter()
    gn, gq = m.adj_backward(None, len(sc.inflow[5]))
    t2 = time.perf_counter()
    m.close()
    return {"grid": f"{nx}x{nx}", "steps": steps, "dt_s": sc.dt_fixed, "gauges": ngauges,
            "observations": steps // obs_every, "checkpoints": int(np.ceil(steps / np.ceil(np.sqrt(steps)))),
            "loss": loss, "grad_n_nonzero": int((gn != 0).sum()), "grad_q_norm": float(np.linalg.norm(gq)),
            "forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
            "adjoint_gcell_s": round(cells * steps / (t2 - t0) / 1e9, 3),
            "plain_tiling_autotuned": list(best),
            "plain_gcell_s": round(cells * steps / (plain_ms / 1e3) / 1e9, 3),
            "adjoint_vs_plain": round((plain_ms / 1e3) / (t2 - t0), 4),
            "plain_two_step_gcell_s": round(cells * steps / (plain2_ms / 1e3) / 1e9, 3),
            "plain_three_step_gcell_s": round(cells * steps / (plain3_ms / 1e3) / 1e9, 3),
            "adjoint_vs_best_plain": round((min(plain_ms, plain2_ms, plain3_ms) / 1e3) / (t2 - t0), 4)}


# (cells per lane, rows per work item) the active-tile autotuner tries: small
# items when few hold water (the march of one item is then the step's
# critical path), large ones when many do
ACTIVE_TILINGS = [(4, 32), (4, 16), (2, 16), (4, 8), (2, 8), (1, 8)]


def run_active(fl, torch, sc, warmup: int, steps: int, full_value: float, full_depth=None,
               sample_every: int = 50):
    """The same workload with active-tile skipping.  On the state after the
    warm-up, outside the timed region, the autotuners pick the single-step
    tiling and then one or three steps per launch, both by skipping trial steps.
    Reports the time per step, the work items computed (read back every
    `sample_every` steps in a second, untimed run) and whether the final depth
    equals that of the run that computes every item."""
    cells = sc.nx * sc.ny
    stream = torch.cuda.current_stream().cuda_stream
    f = fl.from_scenario(sc, "f32", device=0, stream=stream, active_tiles=True, fusion=3)
    f.step(warmup)
    best, _ = f.autotune(ACTIVE_TILINGS, 20)
    spl, _ = f.autotune_fusion(20)
    torch.cuda.synchronize()
    ms = f.time_steps(steps)
    end_items, total = f.active_items()
    rep = f.get_report()
    same = None
    if full_depth is not None:
        h = torch.empty_like(full_depth)
        f.get_depth(h)
        same = bool(torch.equal(h, full_depth))
        del h
    f.close()
    progress("active tiles: timed; sampling computed items")
    g = fl.from_scenario(sc, "f32", device=0, stream=stream, active_tiles=True,
                         cells_per_lane=best[0], rows_per_item=best[1], fusion=spl)
    g.step(warmup)
    counts = []
    every = max(1, min(sample_every, steps))
    for _ in range(steps // every):
        g.step(every)
        counts.append(g.active_items()[0])
    g.close()
    value = cells * steps / (ms / 1e3) / 1e9
    return {"steps_per_launch_autotuned": spl, "single_step_tiling_autotuned": list(best),
            "ms_per_step": round(ms / steps, 5),
            "gcell_s_grid_equivalent": round(value, 3),
            "vs_full_grid_headline": round(value / full_value, 2),
            "items_per_step": total, "items_computed_last_step": end_items,
            "items_computed_mean_sampled": (round(float(sum(counts)) / len(counts), 1)
                                            if counts else None),
            "sample_every_steps": every,
            "same_depth_as_full_grid": same, "budget_error": rep.budget_error()}


def run_variants(fl, torch, steps: int = 20000, nx: int = 2048):
    """How much two readings of the paper matter: the 2048^2 valley (5 m, the
    triangular 500 m^3/s hydrograph, 20000 CFL steps) under the default
    method and each variant (vector-norm friction; literal cell-area Manning
    boundaries; both): flooded area (h > 0.1 m), deepest cell, outflow volume,
    and the step rate of each variant's kernel (one step per launch)."""
    import numpy as np
    import synth
    sc = synth.config_d2(nx, steps)
    stream = torch.cuda.current_stream().cuda_stream
    cells = nx * nx
    out = {"grid": f"{nx}x{nx}", "dx_m": sc.dx, "steps": steps, "threshold_m": 0.1}
    base = None
    for name, var in (("default", ("face", "section")), ("friction_vector", ("vector", "section")),
                      ("boundary_cell_area", ("face", "cell_area")),
                      ("both", ("vector", "cell_area"))):
        f = fl.from_scenario(sc, "f32", device=0, stream=stream, variant=var)
        ms = f.time_steps(steps)
        h = f.get_depth()
        r = f.get_report()
        f.close()
        wet = h > 0.1
        d = {"flooded_km2": round(float(wet.sum()) * sc.dx * sc.dx / 1e6, 4),
             "max_depth_m": round(float(h.max()), 4), "v_out_m3": round(r.v_out, 1),
             "sim_time_s": round(r.t, 1), "budget_error": r.budget_error(),
             "gcell_s": round(cells * steps / (ms / 1e3) / 1e9, 2)}
        if base is None:
            base = (wet, h)
        else:
            d["flooded_cells_differing_from_default"] = int(np.count_nonzero(wet != base[0]))
            d["max_abs_depth_difference_m"] = round(float(np.abs(h - base[1]).max()), 4)
        out[name] = d
    return out


def run_sweep(fl, torch, steps: int = 4000, nx: int = 1024, members: int = 16):
    """Flooded extent against discharge: one 1024^2 valley at 5 m, constant inflows
    from 25 to 1600 m^3/s (geometric), fixed dt 0.25 s; the members run in one
    batched launch or one after another, whichever frozen trials find faster."""
    import numpy as np
    import synth
    from paper_2204_10323_amd.sweep import discharge_sweep
    v = synth.Valley(nx, nx, 5.0, 5e-4, 2.0, 40.0, 0.3, seed=2, meander=True)
    z = synth._f32(synth.valley_dem64(v))
    n = synth._f32(synth.manning_field(v))
    first, count = synth.west_section(v, 40.0)
    qs = [float(q) for q in np.geomspace(25.0, 1600.0, members)]
    out = discharge_sweep(z, n, v.dx, (synth.WEST, first, count, 5e-4),
                          (synth.EAST, 0, nx, 5e-4), qs, steps, 0.25,
                          stream=torch.cuda.current_stream().cuda_stream)
    progress("discharge sweep: members one after another with active tiles")
    act = discharge_sweep(z, n, v.dx, (synth.WEST, first, count, 5e-4),
                          (synth.EAST, 0, nx, 5e-4), qs, steps, 0.25, mode="sequential",
                          active_tiles=True, stream=torch.cuda.current_stream().cuda_stream)
    cells = nx * nx * members
    gcell = cells * steps / (out["ms"] / 1e3) / 1e9
    gcell_act = cells * steps / (act["ms"] / 1e3) / 1e9
    return {"grid": f"{nx}x{nx}", "dx_m": 5.0, "members": members, "steps": steps,
            "simulated_s": out["seconds"], "threshold_m": out["threshold"],
            "discharge_m3s": [round(q, 1) for q in qs],
            "flooded_km2": [round(a / 1e6, 4) for a in out["flooded_area_m2"]],
            "max_depth_m": [round(float(h), 3) for h in out["max_depth"]],
            "max_budget_error": float(out["budget_error"].max()),
            "mode": out["mode"],
            "steps_per_entry": out["steps_per_entry"],
            "gcell_s": round(gcell, 3),
            "active_tiles_gcell_s_grid_equivalent": round(gcell_act, 3),
            "active_tiles_vs_gcell_s": round(gcell_act / gcell, 2),
            "active_tiles_same_results": bool(
                np.array_equal(act["flooded_cells"], out["flooded_cells"]) and
                np.array_equal(act["max_depth"], out["max_depth"]) and
                np.array_equal(act["v_in"], out["v_in"]) and
                np.allclose(act["v_out"], out["v_out"], rtol=1e-13, atol=0.0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="valley16384_wet", choices=sorted(WORKLOAD_NAMES),
                    help="valley16384_wet: pre-wetted start (default); valley16384: dry start")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--fusion", type=int, default=3, choices=[1, 2, 3],
                    help="time steps per launch (3: three chained steps per launch, the default)")
    ap.add_argument("--cells-per-lane", type=int, default=0,
                    help="tiling of the kernel in use (0: its default)")
    ap.add_argument("--rows-per-item", type=int, default=0)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the other steps-per-launch setting for comparison")
    ap.add_argument("--steps-per-graph", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-other-start", action="store_true",
                    help="skip the other start of the same grid (dry start when the headline is "
                         "pre-wetted, and the reverse)")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the batched-ensemble comparison (64 uneven grids)")
    ap.add_argument("--ensemble-steps", type=int, default=5000)
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the discharge sweep (16 discharges on a 1024^2 valley, one batch)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the method-variant comparison (2048^2 valley, 20000 steps each)")
    ap.add_argument("--no-active", action="store_true",
                    help="skip the same workloads with active-tile (wet-region) skipping")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint comparison (1024^2, 5000 steps)")
    ap.add_argument("--copy-gib", type=float, default=16.0,
                    help="size of the plain streams that measure the copy ceilings (0: skip)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the flood step runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the step is not sharded over several GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2204_10323_amd as fl

    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    sc, wname = build_workload(args.workload)
    t_gen = time.perf_counter() - t_gen
    cells = sc.nx * sc.ny
    stream = torch.cuda.current_stream().cuda_stream
    f32 = args.precision == "f32"

    def run_timed(scn, fusion=args.fusion, keep_depth=False):
        tiling = dict(cells_per_lane=args.cells_per_lane, rows_per_item=args.rows_per_item)
        if fusion >= 2:
            tiling = dict(fusion=(fusion, args.cells_per_lane, args.rows_per_item))
        f = fl.from_scenario(scn, args.precision, device=0, stream=stream,
                             steps_per_graph=args.steps_per_graph, **tiling)
        try:
            f.step(args.warmup)
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            ev_ms = f.time_steps(args.steps)     # HIP events on the stream the kernel runs on
            torch.cuda.synchronize()
            wall = time.perf_counter() - w0
            rep = f.get_report()
            dev_bytes = f.device_bytes()
            depth = None
            if keep_depth:
                depth = torch.empty((scn.ny, scn.nx), dtype=torch.float32 if f32 else torch.float64,
                                    device="cuda")
                f.get_depth(depth)
        finally:
            f.close()
        return ev_ms, wall, rep, dev_bytes, depth

    def gcell(ms):
        return round(cells * args.steps / (ms / 1e3) / 1e9, 3)

    progress(f"inputs ready ({t_gen:.1f} s); timing {args.steps} steps of {wname}")
    keep = not args.no_active and f32
    ev_ms, wall, rep, dev_bytes, full_depth = run_timed(sc, keep_depth=keep)
    progress(f"timed: {ev_ms / args.steps:.4f} ms/step")
    ms_step = ev_ms / args.steps
    value = cells * args.steps / (ev_ms / 1e3) / 1e9
    bpc = BYTES_PER_CELL[args.precision]
    # Roofline of the dominant kernel.  One launch makes `fusion` steps but
    # reads the state (h, z, n, qx, qy) once and writes it (h, qx, qy) once:
    # its algorithmic bytes are one pass, bpc x cells, whatever the steps per
    # launch.  Its duration: the timed region over the working launches (the
    # region also holds the launch that settles the last speculated step and
    # the read-back of the step count, so this slightly overstates it).
    launches = max(1, -(-args.steps // args.fusion))
    launch_ms = ev_ms / launches
    alg_bytes = bpc * cells
    achieved = alg_bytes / (launch_ms / 1e3) / 1e9
    traffic = measured_traffic(cells, args.fusion, wname) if f32 else None
    out = {
        "metric": "Gcell-updates/s + % of HBM BW; batched & adjoint vs plain step, same GPU",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": wname, "grid": f"{sc.nx}x{sc.ny}", "dx_m": sc.dx,
                   "cells": cells, "dt": "CFL alpha 0.7, device-side", "dt_max_s": sc.dt_max,
                   "inflow_cells": sc.inflow[2], "outflow": "east edge",
                   "steps_per_launch": args.fusion,
                   "steps_in_run": args.warmup + args.steps, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "steps_per_launch": args.fusion,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "launches_timed": launches,
                     "launch_ms": round(launch_ms, 5),
                     # the bytes the launch actually moves (PMC), as a fraction of the peak
                     "traffic_frac": (round(traffic / (launch_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic else None),
                     # what a kernel making one pass per step would have to move
                     # for the same rate: a cell-update equivalent, not HBM bytes
                     "one_pass_per_step_equivalent_gbs": round(achieved * args.fusion, 1),
                     # SQ counters of the same kernel (committed profile, current sources
                     # only): the fraction of cycles its SIMDs issue VALU instructions
                     "valu_busy": measured_valu_busy(args.fusion) if f32 else None},
    }
    extras = {"wall_s_timed_region": round(wall, 4), "input_generation_s": round(t_gen, 1),
              "device_bytes": dev_bytes, "budget_error": rep.budget_error(),
              "sim_time_s": rep.t, "kernel_sha256_16": kernel_hash()}
    others = [k for k in (1, 2, 3) if k != args.fusion]
    if not args.no_compare:
        for other in others:
            ev1, _, rep1, _, _ = run_timed(sc, other)
            extras[f"steps_per_launch_{other}_gcell_s"] = gcell(ev1)
            extras[f"steps_per_launch_{other}_same_clock"] = (rep1.t == rep.t and
                                                               rep1.steps == rep.steps)
    if keep:
        progress("active tiles")
        extras["active_tiles"] = run_active(fl, torch, sc, args.warmup, args.steps, value, full_depth)
    del full_depth
    if not args.no_other_start:
        import synth
        oname = "valley16384" if args.workload == "valley16384_wet" else "valley16384_wet"
        key = "dry_start" if oname == "valley16384" else "prewetted"
        progress(f"{key}: same grid")
        del sc
        sco, _ = build_workload(oname)
        d = {"workload": WORKLOAD_NAMES[oname]}
        keep_o = not args.no_active and f32
        ev2, _, rep2, _, depth_o = run_timed(sco, args.fusion, keep_depth=keep_o)
        d[f"steps_per_launch_{args.fusion}_gcell_s"] = gcell(ev2)
        d["budget_error"] = rep2.budget_error()
        if not args.no_compare:
            for other in others:
                ev3, _, _, _, _ = run_timed(sco, other)
                d[f"steps_per_launch_{other}_gcell_s"] = gcell(ev3)
        if keep_o:
            d["active_tiles"] = run_active(fl, torch, sco, args.warmup, args.steps,
                                           cells * args.steps / (ev2 / 1e3) / 1e9, depth_o)
        del depth_o, sco
        extras[key] = d
        sc = None
    if not args.no_ensemble:
        progress("ensemble")
        extras["ensemble"] = run_ensemble(fl, torch, args.ensemble_steps)
    if not args.no_adjoint:
        progress("adjoint")
        extras["adjoint"] = run_adjoint(fl, torch)
    if not args.no_sweep:
        progress("discharge sweep")
        extras["discharge_sweep"] = run_sweep(fl, torch)
    if not args.no_variants:
        progress("method variants")
        extras["method_variants"] = run_variants(fl, torch)
    if args.copy_gib > 0:
        progress("copy ceilings")
        torch.cuda.empty_cache()
        nbytes = int(args.copy_gib * (1 << 30))
        cc = {"bytes": nbytes,
              "kernel_copy_gbs": round(probe_stream(nbytes, 10, 1), 1),
              "hip_memcpy_d2d_gbs": round(probe_stream(nbytes, 10, 7), 1),
              "read_only_gbs": round(probe_stream(nbytes, 10, 4), 1),
              "write_only_gbs": round(probe_stream(nbytes, 10, 5), 1)}
        best_copy = max(cc["kernel_copy_gbs"], cc["hip_memcpy_d2d_gbs"])
        cc["step_launch_traffic_vs_best_copy"] = (
            round(traffic / (launch_ms / 1e3) / 1e9 / best_copy, 4) if traffic else None)
        cc["step_launch_algorithmic_vs_best_copy"] = round(achieved / best_copy, 4)
        extras["copy_ceilings"] = cc
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        if sc is None:
            sc, _ = build_workload(args.workload)
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_budget)
        extras["cpu_oracle_single_thread"] = cpu_single_thread(sc)
    out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
