"""Flooded extent against inflow discharge (the paper's extent-versus-discharge
study, Results: flood extents for a range of river discharges), with every
discharge of the sweep a member of one batched, persistent launch.

All members share one DEM, roughness field and boundary sections and differ
only in the constant inflow Q.  They run the paper's constant-dt mode (Methods:
a fixed time step), so every member reaches the same simulated time after the
same number of steps.  A cell counts as flooded when its depth exceeds
`threshold` metres.
"""
from typing import Optional, Sequence

import numpy as np

from . import Batch, Flood

# (cells per lane, rows per work item) the autotuners try: for the batch
# launch, and for one member stepped alone
BATCH_TILINGS = [(4, 8), (4, 16), (4, 32), (4, 64), (2, 16), (2, 32), (1, 16)]
SINGLE_TILINGS = [(1, 4), (1, 8), (2, 4), (2, 8), (4, 8), (4, 16), (4, 32)]
# ... and for a batch launch with several steps per queue entry
MULTI_TILINGS = [(2, 16), (2, 32), (2, 64), (1, 32)]


def discharge_sweep(z: np.ndarray, n: np.ndarray, dx: float, inflow_section: tuple,
                    outflow_section: Optional[tuple], discharges: Sequence[float], steps: int,
                    dt: float, threshold: float = 0.1, precision: str = "f32", device: int = 0,
                    stream=None, h0: Optional[np.ndarray] = None, keep_depths: bool = False,
                    tiling: Optional[tuple] = None, trial_steps: int = 10, mode: str = "auto",
                    active_tiles: bool = False, steps_per_entry: int = 0, **params) -> dict:
    """Run one member per discharge (m^3/s) for `steps` steps of `dt` seconds.

    inflow_section: (side, first, count, slope); outflow_section: (side, first,
    count, slope) or None (closed borders).
    mode: "batch" (all members in one persistent launch), "sequential" (one
    member after another, each with its own graph-captured steps) or "auto":
    time both over `trial_steps` frozen steps (which leave the state as it is),
    each with its autotuned tiling, and run the faster.  With only a few
    members per XCD the batch launch has too little independent work to hide
    the wait between a member's steps.
    tiling: (cells_per_lane, rows_per_item) of the batch launch (mode
    "batch"), or None for the autotuner's choice.
    steps_per_entry: steps per queue entry of the batch launch, 1, 2 or 3
    (fl_batch_set_fusion; the members then make the multi-step launches of
    their own runs, bit for bit); 0: 3, or 1 with active tiles.
    active_tiles: the members skip the work items that no water can reach
    (fl_set_active_tiles), in the batch launch and one after another; the
    tilings are then autotuned with skipping trial steps.
    Returns per-member arrays: flooded cell count and area, deepest cell,
    inflow and outflow volume, relative volume-budget error, and the depths if
    keep_depths; the mode used and its time in milliseconds.
    """
    if mode not in ("auto", "batch", "sequential"):
        raise ValueError("discharge_sweep: mode must be auto, batch or sequential")
    if steps < 1 or not (dt > 0.0):
        raise ValueError("discharge_sweep: steps >= 1 and dt > 0 are required")
    if steps_per_entry not in (0, 1, 2, 3):
        raise ValueError("discharge_sweep: steps_per_entry must be 0, 1, 2 or 3")
    if active_tiles and steps_per_entry > 1:
        raise ValueError("discharge_sweep: members with active tiles run one step per queue entry")
    k = steps_per_entry or (1 if active_tiles else 3)
    z = np.ascontiguousarray(z)
    ny, nx = z.shape
    side, first, count, slope = inflow_section
    members = []
    try:
        for q in discharges:
            f = Flood(nx, ny, dx, precision, device, stream)
            members.append(f)
            f.set_dem(z)
            f.set_manning(n)
            f.set_inflow(side, first, count, slope, np.array([0.0]), np.array([float(q)]))
            if outflow_section is not None:
                f.set_outflow(*outflow_section)
            f.set_params(dt_fixed=dt, **params)
            if h0 is not None:
                f.set_state(h0, None, None, 0.0)
            if active_tiles:
                f.set_active_tiles(True)
            if k > 1 and mode != "sequential":
                f.set_fusion(k)   # the buffers of the multi-step launches
            f.commit()
        fp64 = precision in ("f64", "fp64", "double")
        single_cands = [t for t in SINGLE_TILINGS if not fp64 or t[0] < 4]
        ms = 0.0
        if mode == "sequential":
            best, _ = members[0].autotune(single_cands, trial_steps)
        else:
            b = Batch(members)
            try:
                if k > 1:
                    b.set_fusion(k, *(tiling or (0, 0)))
                elif tiling is not None:
                    b.set_tiling(*tiling)
                if tiling is not None:
                    mode = "batch"
                else:
                    cands = MULTI_TILINGS if k > 1 else [t for t in BATCH_TILINGS if not fp64 or t[0] < 4]
                    _, batch_trial = b.autotune(cands, trial_steps)
                    if mode == "auto":
                        # members share the grid: one member's tuned step, times their number
                        best, one = members[0].autotune(single_cands, trial_steps)
                        mode = "sequential" if one * len(members) < batch_trial else "batch"
                if mode == "batch":
                    ms = b.time(steps)
            finally:
                b.close()
        if mode == "sequential":
            # one step per launch, the tuned single-step tiling
            for f in members:
                f.set_fusion(1)
                f.set_tiling(*best)
                f.commit()
            ms = sum(f.time_steps(steps) for f in members)
        out = {"discharge": np.asarray(discharges, dtype=np.float64), "steps": steps, "dt": dt,
               "seconds": steps * dt, "threshold": threshold, "mode": mode, "ms": ms,
               "steps_per_entry": k if mode == "batch" else None,
               "flooded_cells": [], "flooded_area_m2": [], "max_depth": [], "v_in": [],
               "v_out": [], "budget_error": []}
        if keep_depths:
            out["depth"] = []
        for f in members:
            h = f.get_depth()
            r = f.get_report()
            wet = int(np.count_nonzero(h > threshold))
            out["flooded_cells"].append(wet)
            out["flooded_area_m2"].append(wet * dx * dx)
            out["max_depth"].append(float(h.max()))
            out["v_in"].append(r.v_in)
            out["v_out"].append(r.v_out)
            out["budget_error"].append(r.budget_error())
            if keep_depths:
                out["depth"].append(h)
        for k in ("flooded_cells", "flooded_area_m2", "max_depth", "v_in", "v_out", "budget_error"):
            out[k] = np.asarray(out[k])
        return out
    finally:
        for f in members:
            f.close()
