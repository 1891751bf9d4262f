"""Write the expected values of the pre-wetted 16384^2 valley run (dx 1 m,
1000 CFL steps) from the FP64 CPU oracle.  Calls only the oracle and the
seeded input generator.

    python tests/golden/make_d3wet_golden.py     # ~30 min and ~25 GB on 8 cores

The whole 268 M-cell grid is too large to store, so the file keeps the
oracle's depth and face discharges (FP64 values rounded once to float32 for
storage, below 5e-7 of the value) on a lattice of every 64th cell in each
direction and on four dense 256 x 256 blocks: at the inflow section, across
the channel at mid-valley, at the outflow edge, and across the shoreline of
the initial lake; plus the clock, the volume budget and a hash of the inputs.
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

N, STEPS, STRIDE, OFF, B = 16384, 1000, 64, 32, 256


def input_hash(sc) -> str:
    h = hashlib.sha256()
    for a in (sc.z, sc.n, sc.h0):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    side, first, count, slope, ts, qs = sc.inflow
    h.update(np.array([side, first, count], np.int64).tobytes())
    h.update(np.asarray(ts, np.float64).tobytes() + np.asarray(qs, np.float64).tobytes())
    return h.hexdigest()


def block_origins(sc):
    """(row, column) of the four dense blocks."""
    side, first, count, slope, ts, qs = sc.inflow
    mid = sc.ny // 2
    j_in = min(max(first + count // 2 - B // 2, 0), sc.ny - B)
    # the channel's deepest bed across the valley at mid-valley and at the east edge
    j_mid = int(np.argmin(sc.z[:, sc.nx // 2])) - B // 2
    j_out = int(np.argmin(sc.z[:, sc.nx - 1])) - B // 2
    # the first wet-to-dry change along the middle row: the lake's shoreline
    row = sc.h0[mid] > 0
    edges = np.nonzero(row[1:] != row[:-1])[0]
    i_sh = int(edges[0]) if edges.size else sc.nx // 4
    clamp = lambda v, hi: int(min(max(v, 0), hi - B))  # noqa: E731
    return np.array([[j_in, 0],
                     [clamp(j_mid, sc.ny), sc.nx // 2 - B // 2],
                     [clamp(j_out, sc.ny), sc.nx - B],
                     [clamp(mid - B // 2, sc.ny), clamp(i_sh - B // 2, sc.nx)]], dtype=np.int64)


def main():
    sc = synth.config_d3(N, wet=True, steps=STEPS)
    blocks = block_origins(sc)
    o = oracle.Run(sc)
    t0 = time.time()
    for k in range(10):
        o.step(STEPS // 10)
        print(f"{(k + 1) * STEPS // 10} steps, t = {o.clock.t:.1f} s, "
              f"{time.time() - t0:.0f} s wall", flush=True)
    lat = (slice(OFF, None, STRIDE), slice(OFF, None, STRIDE))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)  # noqa: E731
    np.savez_compressed(
        os.path.join(HERE, "d3wet_16384_1000.npz"),
        lattice=np.array([STRIDE, OFF]), block_size=np.array(B), block_origin=blocks,
        h_lat=f32(o.h[lat]), qx_lat=f32(o.qx[lat]), qy_lat=f32(o.qy[lat]),
        h_blocks=np.stack([f32(o.h[j:j + B, i:i + B]) for j, i in blocks]),
        qx_blocks=np.stack([f32(o.qx[j:j + B, i:i + B + 1]) for j, i in blocks]),
        qy_blocks=np.stack([f32(o.qy[j:j + B + 1, i:i + B]) for j, i in blocks]),
        qmax=np.array(max(np.abs(o.qx).max(), np.abs(o.qy).max())),
        t=np.array(o.clock.t), steps=np.array(o.clock.steps), v_in=np.array(o.clock.v_in),
        v_out=np.array(o.clock.v_out), v0=np.array(o.v0), volume=np.array(o.volume()),
        hmax=np.array(o.h.max()), input_sha256=np.array(input_hash(sc)))
    print("budget error", o.budget_error())


if __name__ == "__main__":
    main()
