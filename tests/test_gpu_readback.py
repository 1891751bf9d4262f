"""Host read-back and strided device inputs of the C interface on the GPU.

Read-backs into host memory go as 1D copies of whole row blocks through a
bounded staging buffer (64 MiB), then row by row on the host; device inputs of
the setters come back the same way.  These tests check that the values arrive
bitwise: a state written with fl_set_state is read back unchanged, on a grid
whose rows span several staging blocks and whose width is ragged, into packed
and into pitched host arrays, and strided device inputs give the run their
packed host copies give.
"""
import numpy as np
import pytest

import paper_2204_10323_amd as fl
from gpu_util import run_gpu
from synth import random_tiny

pytestmark = pytest.mark.gpu


def _committed_with_state(nx, ny, prec, seed):
    dt = np.float64 if prec == "f64" else np.float32
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.0, 3.0, (ny, nx)).astype(dt)
    qx = rng.uniform(-1.0, 1.0, (ny, nx + 1)).astype(dt)
    qy = rng.uniform(-1.0, 1.0, (ny + 1, nx)).astype(dt)
    f = fl.Flood(nx, ny, 2.0, prec)
    f.set_dem(np.zeros((ny, nx), dt))
    f.set_manning(np.full((ny, nx), 0.03, dt))
    f.set_params(dt_max=0.1)
    f.set_state(h, qx, qy)
    f.commit()
    return f, h, qx, qy


@pytest.mark.parametrize("prec,nx,ny", [("f32", 4100, 8200), ("f64", 1531, 6000)])
def test_state_round_trip_through_staged_readback(prec, nx, ny):
    """The committed state reads back bitwise, packed and pitched.  At 4100 x
    8200 FP32 a padded row is 16.6 KB, so the 8200 rows take three staging
    blocks; at 1531 x 6000 FP64 two."""
    f, h, qx, qy = _committed_with_state(nx, ny, prec, 11)
    try:
        assert np.array_equal(f.get_depth(), h)
        gx, gy = f.get_discharge()
        assert np.array_equal(gx, qx) and np.array_equal(gy, qy)
        # pitched host destination: the columns beyond nx keep their values
        wide = np.full((ny, nx + 37), -7.0, dtype=h.dtype)
        f.get_depth(wide[:, :nx])
        assert np.array_equal(wide[:, :nx], h)
        assert np.all(wide[:, nx:] == -7.0)
    finally:
        f.close()


def test_strided_device_inputs_match_packed_host_inputs():
    """DEM and Manning n given as strided views of wider device tensors (read
    back through the staging path) give bitwise the run of packed host arrays."""
    import torch
    sc = random_tiny(45, 23, 9)
    h_ref, qx_ref, qy_ref, _ = run_gpu(sc, 12, "f32")
    zw = torch.full((sc.ny, sc.nx + 19), 123.0, dtype=torch.float32, device="cuda")
    nw = torch.full((sc.ny, sc.nx + 5), 9.0, dtype=torch.float32, device="cuda")
    zw[:, :sc.nx] = torch.from_numpy(sc.z.astype(np.float32)).cuda()
    nw[:, :sc.nx] = torch.from_numpy(sc.n.astype(np.float32)).cuda()
    f = fl.Flood(sc.nx, sc.ny, sc.dx, "f32")
    f.set_dem(zw[:, :sc.nx])
    f.set_manning(nw[:, :sc.nx])
    side, first, count, slope, ts, qs = sc.inflow
    f.set_inflow(side, first, count, slope, ts, qs)
    f.set_outflow(*sc.outflow)
    f.set_params(dt_max=sc.dt_max)
    f.set_state(sc.h0, sc.extra["qx0"], sc.extra["qy0"])
    f.commit()
    f.step(12)
    h = f.get_depth()
    qx, qy = f.get_discharge()
    f.close()
    assert np.array_equal(h, h_ref)
    assert np.array_equal(qx, qx_ref) and np.array_equal(qy, qy_ref)
