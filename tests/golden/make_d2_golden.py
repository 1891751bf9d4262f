"""Write the expected values of the 2048^2 valley run (20000 CFL steps) from the
FP64 CPU oracle.  Calls only the oracle and the seeded input generator.

    python tests/golden/make_d2_golden.py        # ~20 min on 8 cores

Stores (d2_2048_20000.npz): the depth of every cell (the oracle's FP64 value
rounded once to float32 for storage, an error below 5e-7 m for depths under
10 m, far inside the 1e-3 m gate it is compared at), the clock, the volume
budget, and a hash of the float32 inputs so a changed generator is detected.
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def input_hash(sc) -> str:
    h = hashlib.sha256()
    for a in (sc.z, sc.n):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    side, first, count, slope, ts, qs = sc.inflow
    h.update(np.array([side, first, count], np.int64).tobytes())
    h.update(np.asarray(ts, np.float64).tobytes() + np.asarray(qs, np.float64).tobytes())
    return h.hexdigest()


def main():
    sc = synth.config_d2()
    o = oracle.Run(sc)
    t0 = time.time()
    for k in range(20):
        o.step(sc.steps // 20)
        print(f"{(k + 1) * sc.steps // 20} steps, t = {o.clock.t:.1f} s, "
              f"{time.time() - t0:.0f} s wall", flush=True)
    np.savez_compressed(
        os.path.join(HERE, "d2_2048_20000.npz"),
        h_full=o.h.astype(np.float32),
        t=np.array(o.clock.t), steps=np.array(o.clock.steps), v_in=np.array(o.clock.v_in),
        v_out=np.array(o.clock.v_out), v0=np.array(o.v0), volume=np.array(o.volume()),
        hmax=np.array(o.h.max()), input_sha256=np.array(input_hash(sc)))
    print("budget error", o.budget_error())


if __name__ == "__main__":
    main()
