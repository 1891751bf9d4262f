"""The batched ensemble at its full configuration against the FP64 oracle.

64 synthetic valleys at dx 5 m with sides drawn log-uniformly from [256, 2048]
(each its own DEM, a uniform Manning n in [0.02, 0.08] stored as a field, and
a triangular hydrograph peaking at 50-800 m^3/s), 5000 CFL steps each, FP32,
all in ONE persistent batch launch with the tiling the benchmark's batch
autotuner picks (one step per queue entry; with three steps per entry every
member ends bit for bit the same).  A size-stratified subset of six members, the smallest and
the largest included, is compared cell by cell with the oracle run on the same
float32 inputs: max|dh| <= 1e-3 m (the FP32 gate), the member's FP64 volume
budget <= 1e-6 of the volume that entered, and its clock.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2204_10323_amd as fl
import synth
from gpu_util import max_abs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STEPS = 5000


def test_ensemble_64_members_5000_steps_one_launch_against_oracle():
    sys.path.insert(0, ROOT)
    from bench import BATCH_TILINGS
    print("CASE ensemble gate: generating 64 members", flush=True)
    sizes = synth.ensemble_sizes(64)
    scs = [synth.config_d4_member(s, side, STEPS) for s, side in enumerate(sizes)]
    members = [fl.from_scenario(sc, "f32") for sc in scs]
    b = fl.Batch(members)
    best, _ = b.autotune(BATCH_TILINGS, 20)
    print(f"CASE ensemble gate: one batch launch of {STEPS} steps, tiling {best}", flush=True)
    b.run(STEPS)
    b.close()
    order = np.argsort(sizes, kind="stable")
    pick = [int(order[k]) for k in np.linspace(0, len(sizes) - 1, 6).round().astype(int)]
    assert sizes[pick[0]] == min(sizes) and sizes[pick[-1]] == max(sizes)
    for f in members:
        r = f.get_report()
        assert r.steps == STEPS and r.budget_error() <= 1e-6
    # the benchmark's fastest batch configuration, three steps per queue entry,
    # gives every member bit for bit the state checked against the oracle below
    from bench import BATCH2_TILINGS
    members3 = [fl.from_scenario(sc, "f32", fusion=3) for sc in scs]
    b3 = fl.Batch(members3)
    b3.set_fusion(3)
    best3, _ = b3.autotune(BATCH2_TILINGS, 20)
    print(f"CASE ensemble gate: three steps per queue entry, tiling {best3}", flush=True)
    b3.run(STEPS)
    b3.close()
    for s, (f, g) in enumerate(zip(members, members3)):
        r, r3 = f.get_report(), g.get_report()
        assert np.array_equal(f.get_depth(), g.get_depth()), f"member {s}"
        assert r3.steps == r.steps and r3.t == r.t and r3.v_in == r.v_in, f"member {s}"
        g.close()
    for s in pick:
        sc, f = scs[s], members[s]
        h = f.get_depth()
        r = f.get_report()
        print(f"CASE ensemble gate: member {s} ({sc.nx}x{sc.ny}) against the oracle", flush=True)
        o = oracle.Run(sc)
        o.step(STEPS)
        err = max_abs(h, o.h)
        print(f"member {s} {sc.nx}x{sc.ny}: max|dh| = {err:.3e} m, max h = {o.h.max():.3f} m, "
              f"wet cells {(o.h > 0.01).sum()}, budget {r.budget_error():.2e}", flush=True)
        assert (o.h > 0.05).sum() > 100, "the member must have flooded"
        assert err <= 1e-3
        assert o.clock.steps == STEPS
        assert abs(r.t / o.clock.t - 1) <= 1e-5
        assert abs(r.v_in / o.clock.v_in - 1) <= 1e-5
        assert o.budget_error() <= 1e-12
    for f in members:
        f.close()
