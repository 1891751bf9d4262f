"""Helpers shared by the GPU parity tests: run a scenario through libflood and
through the FP64 oracle from the same float32 inputs, and compare."""
import numpy as np

import oracle
import paper_2204_10323_amd as fl


def run_gpu(sc, steps, precision="f32", cells_per_lane=0, rows_per_item=0, **params):
    f = fl.from_scenario(sc, precision, cells_per_lane=cells_per_lane,
                         rows_per_item=rows_per_item, **params)
    f.step(steps)
    h = f.get_depth()
    qx, qy = f.get_discharge()
    r = f.get_report()
    f.close()
    return h, qx, qy, r


def run_oracle(sc, steps, **kw):
    o = oracle.Run(sc, **kw)
    o.step(steps)
    return o


def rel_err(a, b):
    """max|a-b| / max(max|b|, tiny)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / s)


def max_abs(a, b):
    return float(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).max())
