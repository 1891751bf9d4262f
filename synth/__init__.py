"""Seeded synthetic inputs for the flood step: valley DEMs, Manning fields,
inflow hydrographs and boundary sections.

This module is shared by the tests, the benchmark and anything that feeds the
CPU oracle or the GPU library.  It holds none of the method's arithmetic (no
face flux, no boundary solve, no depth update): only terrain, roughness and
forcing, generated in float64 and rounded once to float32 so that both sides
of every comparison start from the same bits.

The paper's terrain (a 1 m LiDAR DEM of a river valley, Data section) is not
available, so a valley of the same character stands in for it: a planar
down-valley slope, a Gaussian river channel (straight or meandering) and
seeded fractal value noise.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# Boundary sides, in the order the C interface numbers them.
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def _lattice(seed: int, octave: int, ni: int, nj: int) -> np.ndarray:
    """Hash values in [-1, 1) on an (nj, ni) integer lattice."""
    I = np.arange(ni, dtype=np.uint64)[None, :]
    J = np.arange(nj, dtype=np.uint64)[:, None]
    key = ((np.uint64(seed & 0xFFFF) << np.uint64(48))
           ^ (np.uint64(octave & 0xFF) << np.uint64(40))
           ^ (J << np.uint64(20)) ^ I)
    u = (splitmix64(key) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def _smooth(f: np.ndarray) -> np.ndarray:
    return f * f * (3.0 - 2.0 * f)


def _nthreads() -> int:
    import os
    return max(1, min(16, os.cpu_count() or 1))


def value_noise(nx: int, ny: int, seed: int, octaves: int = 6, base: float = 64.0,
                persistence: float = 0.5) -> np.ndarray:
    """Fractal value noise on an ny x nx raster, normalised to max|N| = 1.

    Octave o has wavelength base/2**o cells and amplitude persistence**o; each
    octave interpolates SplitMix64 lattice values with smoothstep-bilinear
    weights at the cell centres.
    """
    out = np.zeros((ny, nx), dtype=np.float64)
    plan = []
    for o in range(octaves):
        lam = base / (2.0 ** o)
        u = (np.arange(nx, dtype=np.float64) + 0.5) / lam
        v = (np.arange(ny, dtype=np.float64) + 0.5) / lam
        I = np.floor(u).astype(np.int64)
        J = np.floor(v).astype(np.int64)
        lat = _lattice(seed, o, int(I.max()) + 2, int(J.max()) + 2)
        plan.append((persistence ** o, I, _smooth(u - I), J, _smooth(v - J), lat))

    def rows(j0: int, j1: int) -> None:
        acc = out[j0:j1]
        for amp, I, sx, J, sy, lat in plan:
            Jb, syb = J[j0:j1, None], sy[j0:j1, None]
            a = lat[Jb, I[None, :]]
            b = lat[Jb, I[None, :] + 1]
            c = lat[Jb + 1, I[None, :]]
            d = lat[Jb + 1, I[None, :] + 1]
            top = a + (b - a) * sx[None, :]
            bot = c + (d - c) * sx[None, :]
            acc += amp * (top + (bot - top) * syb)

    blk = max(1, min(ny, (1 << 22) // max(nx, 1)))
    spans = [(j, min(ny, j + blk)) for j in range(0, ny, blk)]
    if len(spans) > 1:
        with ThreadPoolExecutor(_nthreads()) as ex:
            list(ex.map(lambda s: rows(*s), spans))
    else:
        rows(0, ny)
    m = float(np.abs(out).max())
    if m > 0:
        out /= m
    return out


@dataclass
class Valley:
    """Parameters of one synthetic valley (all lengths in metres)."""
    nx: int
    ny: int
    dx: float
    slope: float
    depth: float          # channel depth D
    width: float          # channel full width at half maximum w
    noise: float          # noise amplitude A
    seed: int
    meander: bool = False
    n_channel: float = 0.03
    n_plain: float = 0.05


def centreline(v: Valley, x: np.ndarray) -> np.ndarray:
    """Channel centreline y_c(x)."""
    ly = v.ny * v.dx
    if not v.meander:
        return np.full_like(x, (v.ny // 2 + 0.5) * v.dx)
    lx = v.nx * v.dx
    return ly / 2 + 0.1 * ly * np.sin(2 * np.pi * x / (lx / 2))


def channel_distance(v: Valley) -> np.ndarray:
    """Signed distance d = y - y_c(x) of every cell centre, shape (ny, nx)."""
    x = (np.arange(v.nx, dtype=np.float64) + 0.5) * v.dx
    y = (np.arange(v.ny, dtype=np.float64) + 0.5) * v.dx
    return y[:, None] - centreline(v, x)[None, :]


def valley_dem64(v: Valley) -> np.ndarray:
    """z = S*(Lx - x) - D*exp(-d^2/(2 sigma^2)) + A*N, shifted so min z = 0 (float64)."""
    x = (np.arange(v.nx, dtype=np.float64) + 0.5) * v.dx
    d = channel_distance(v)
    sigma = v.width / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    z = v.slope * (v.nx * v.dx - x)[None, :] - v.depth * np.exp(-(d * d) / (2 * sigma * sigma))
    if v.noise:
        z += v.noise * value_noise(v.nx, v.ny, v.seed)
    z -= z.min()
    return z


def manning_field(v: Valley) -> np.ndarray:
    """Per-cell Manning n: channel value where |d| <= w/2, floodplain value elsewhere."""
    d = channel_distance(v)
    return np.where(np.abs(d) <= v.width / 2, v.n_channel, v.n_plain)


def upsample_bilinear(a: np.ndarray, factor: int) -> np.ndarray:
    """Bilinear resampling of cell-centred values onto a grid `factor` times finer."""
    ny, nx = a.shape

    def axis(n: int) -> Tuple[np.ndarray, np.ndarray]:
        s = (np.arange(n * factor, dtype=np.float64) + 0.5) / factor - 0.5
        s = np.clip(s, 0.0, n - 1.0)
        i0 = np.minimum(np.floor(s).astype(np.int64), n - 2) if n > 1 else np.zeros(s.shape, np.int64)
        return i0, s - i0

    ix, fx = axis(nx)
    jy, fy = axis(ny)
    out = np.empty((ny * factor, nx * factor), dtype=np.float64)

    def rows(j0: int, j1: int) -> None:
        J, F = jy[j0:j1, None], fy[j0:j1, None]
        top = a[J, ix[None, :]] * (1 - fx) + a[J, ix[None, :] + 1] * fx
        bot = a[J + 1, ix[None, :]] * (1 - fx) + a[J + 1, ix[None, :] + 1] * fx
        out[j0:j1] = top * (1 - F) + bot * F

    blk = max(1, (1 << 22) // (nx * factor))
    spans = [(j, min(ny * factor, j + blk)) for j in range(0, ny * factor, blk)]
    with ThreadPoolExecutor(_nthreads()) as ex:
        list(ex.map(lambda s: rows(*s), spans))
    return out


@dataclass
class Scenario:
    """Everything one run needs, in the units and conventions of the C interface.

    z, n: float32 (ny, nx).  h0: float32 (ny, nx) initial depth.
    inflow: (side, first, count, slope, t_samples[s], q_samples[m^3/s]) or None.
    outflow: (side, first, count, slope) or None.
    """
    name: str
    nx: int
    ny: int
    dx: float
    z: np.ndarray
    n: np.ndarray
    h0: np.ndarray
    inflow: Optional[tuple]
    outflow: Optional[tuple]
    dt_max: float
    alpha: float = 0.7
    h_eps: float = 1e-4
    g: float = 9.81
    dt_fixed: float = 0.0
    t_end: float = math.inf
    steps: int = 0
    extra: dict = field(default_factory=dict)

    def params(self) -> dict:
        return dict(g=self.g, alpha=self.alpha, dt_max=self.dt_max, h_eps=self.h_eps,
                    dt_fixed=self.dt_fixed, t_end=self.t_end)


def triangle_hydrograph(t_end: float, peak: float, base: float, t_peak: float,
                        every: float) -> Tuple[np.ndarray, np.ndarray]:
    """Triangular hydrograph base -> peak (at t_peak) -> base (at 3 t_peak), sampled every `every` s."""
    t = np.arange(0.0, t_end + every * 0.5, every)
    q = np.where(t <= t_peak, base + (peak - base) * t / t_peak,
                 np.maximum(base, peak - (peak - base) * (t - t_peak) / (2 * t_peak)))
    return t, q


def west_section(v: Valley, halfwidth: float) -> Tuple[int, int]:
    """Rows of the west edge whose centre lies within `halfwidth` of the channel."""
    d = channel_distance(v)[:, 0]
    rows = np.nonzero(np.abs(d) <= halfwidth + 1e-9)[0]
    return int(rows[0]), int(rows[-1] - rows[0] + 1)


def fraction_section(length: int, f_start: float, f_end: float) -> Tuple[int, int]:
    """(first, count) of the cells along a side whose centre fraction (k+1/2)/L is in [f_start, f_end]."""
    k = np.arange(length)
    sel = np.nonzero(((k + 0.5) / length >= f_start) & ((k + 0.5) / length <= f_end))[0]
    if sel.size == 0:
        return 0, 0
    return int(sel[0]), int(sel.size)


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def config_d1() -> Scenario:
    """256^2, dx 10 m, straight channel, 100 m^3/s over 5 west cells, 2000 steps."""
    v = Valley(256, 256, 10.0, 1e-3, 2.0, 30.0, 0.5, seed=1)
    z = _f32(valley_dem64(v))
    n = _f32(manning_field(v))
    first, count = 126, 5
    ts, qs = np.array([0.0]), np.array([100.0])
    return Scenario("d1_256", 256, 256, 10.0, z, n, np.zeros_like(z),
                    (WEST, first, count, 1e-3, ts, qs), (EAST, 0, 256, 1e-3),
                    dt_max=1.0, steps=2000)


def config_d2(nx: int = 2048, steps: int = 20000) -> Scenario:
    """2048^2, dx 5 m, meandering channel, triangular hydrograph peaking at 500 m^3/s."""
    v = Valley(nx, nx, 5.0, 5e-4, 2.0, 40.0, 0.3, seed=2, meander=True)
    z = _f32(valley_dem64(v))
    n = _f32(manning_field(v))
    first, count = west_section(v, 40.0)
    ts, qs = triangle_hydrograph(12000.0, 500.0, 20.0, 3000.0, 60.0)
    return Scenario(f"d2_{nx}", nx, nx, 5.0, z, n, np.zeros_like(z),
                    (WEST, first, count, 5e-4, ts, qs), (EAST, 0, nx, 5e-4),
                    dt_max=0.5, steps=steps)


def config_d3(nx: int = 16384, wet: bool = False, steps: int = 1000) -> Scenario:
    """16384^2 at 1 m: the 2048^2 generator at 8 m upsampled x8 plus fine noise.

    `nx` must be a multiple of 8; smaller values give the same construction at
    a smaller size (used for tests).  `wet` pre-fills the valley to the 30th
    percentile of z ("bathtub" start) so that every cell carries water.
    """
    assert nx % 8 == 0
    coarse = Valley(nx // 8, nx // 8, 8.0, 5e-4, 2.0, 40.0, 0.3, seed=3, meander=True)
    z = upsample_bilinear(valley_dem64(coarse), 8)
    z += 0.05 * value_noise(nx, nx, 33, base=32.0)
    z -= z.min()
    fine = Valley(nx, nx, 1.0, 5e-4, 2.0, 40.0, 0.0, seed=3, meander=True)
    n = _f32(manning_field(fine))
    z32 = _f32(z)
    del z
    if wet:
        eta0 = float(np.percentile(z32[:: max(1, nx // 1024), :: max(1, nx // 1024)], 30))
        h0 = np.maximum(np.float32(eta0) - z32, np.float32(0)).astype(np.float32)
    else:
        h0 = np.zeros_like(z32)
    first, count = west_section(fine, 40.0)
    ts, qs = triangle_hydrograph(3000.0, 500.0, 20.0, 1000.0, 10.0)
    return Scenario(f"d3_{nx}{'_wet' if wet else ''}", nx, nx, 1.0, z32, n, h0,
                    (WEST, first, count, 5e-4, ts, qs), (EAST, 0, nx, 5e-4),
                    dt_max=0.1, steps=steps)


def ensemble_sizes(count: int = 64, seed: int = 4, lo: int = 256, hi: int = 2048) -> List[int]:
    """Square grid sides drawn log-uniformly from [lo, hi] (left ragged)."""
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(count)]


def config_d4_member(s: int, side: int, steps: int = 5000, seed: int = 4) -> Scenario:
    """Ensemble member s: its own DEM (seed 1000+s), uniform Manning n and hydrograph peak."""
    rng = np.random.default_rng([seed, s])
    n_s = float(rng.uniform(0.02, 0.08))
    peak = float(rng.uniform(50.0, 800.0))
    v = Valley(side, side, 5.0, 5e-4, 2.0, 40.0, 0.3, seed=1000 + s, meander=True)
    z = _f32(valley_dem64(v))
    n = np.full((side, side), n_s, dtype=np.float32)
    first, count = west_section(v, 40.0)
    horizon = steps * 0.5
    ts, qs = triangle_hydrograph(horizon, peak, 0.1 * peak, horizon / 3, horizon / 50)
    return Scenario(f"d4_{s}_{side}", side, side, 5.0, z, n, np.zeros_like(z),
                    (WEST, first, count, 5e-4, ts, qs), (EAST, 0, side, 5e-4),
                    dt_max=0.5, steps=steps, extra=dict(n_s=n_s, peak=peak))


def config_d5(nx: int = 1024, steps: int = 5000) -> Scenario:
    """1024^2 at 5 m with fixed dt 0.25 s; 100-sample triangular hydrograph (adjoint workload)."""
    v = Valley(nx, nx, 5.0, 5e-4, 2.0, 40.0, 0.3, seed=5, meander=True)
    z = _f32(valley_dem64(v))
    n = _f32(manning_field(v))
    first, count = west_section(v, 40.0)
    dt = 0.25
    horizon = steps * dt
    ts = np.linspace(0.0, horizon, 100)
    t_peak = 400.0 * horizon / 1250.0
    qs = np.where(ts <= t_peak, 20.0 + 280.0 * ts / t_peak,
                  np.maximum(20.0, 300.0 - 280.0 * (ts - t_peak) / (horizon - t_peak)))
    n_true = _f32(n.astype(np.float64) * (1.0 + 0.2 * value_noise(nx, nx, 56)))
    return Scenario(f"d5_{nx}", nx, nx, 5.0, z, n, np.zeros_like(z),
                    (WEST, first, count, 5e-4, ts, qs), (EAST, 0, nx, 5e-4),
                    dt_max=dt, dt_fixed=dt, steps=steps, extra=dict(n_true=n_true))


def random_tiny(nx: int, ny: int, seed: int, wet_fraction: float = 0.6,
                with_bc: bool = True) -> Scenario:
    """A tiny grid with random terrain, roughness and a random wet/dry state.

    Depths are a mix of exact zeros, tiny films and O(1 m) water; discharges
    are random on wet faces.  Used for step-by-step brute-force comparisons.
    """
    rng = np.random.default_rng(seed)
    z = _f32(rng.uniform(0.0, 2.0, (ny, nx)))
    n = _f32(rng.uniform(0.02, 0.08, (ny, nx)))
    kind = rng.random((ny, nx))
    h = np.where(kind < 1 - wet_fraction, 0.0,
                 np.where(kind < 1 - wet_fraction / 2, rng.uniform(0, 1e-3, (ny, nx)),
                          rng.uniform(0.05, 1.5, (ny, nx))))
    h0 = _f32(h)
    qx = _f32(rng.normal(0, 0.3, (ny, nx + 1)))
    qy = _f32(rng.normal(0, 0.3, (ny + 1, nx)))
    inflow = outflow = None
    if with_bc:
        side_in = int(rng.integers(0, 4))
        side_out = [EAST, WEST, NORTH, SOUTH][side_in]
        L_in = ny if side_in in (WEST, EAST) else nx
        L_out = ny if side_out in (WEST, EAST) else nx
        c_in = int(rng.integers(1, L_in + 1))
        f_in = int(rng.integers(0, L_in - c_in + 1))
        c_out = int(rng.integers(1, L_out + 1))
        f_out = int(rng.integers(0, L_out - c_out + 1))
        ts = np.array([0.0, 5.0, 20.0])
        qs = rng.uniform(0.0, 5.0, 3) * max(nx, ny)
        inflow = (side_in, f_in, c_in, 1e-3, ts, qs)
        outflow = (side_out, f_out, c_out, 1e-3)
    s = Scenario(f"tiny_{nx}x{ny}_{seed}", nx, ny, 1.0, z, n, h0, inflow, outflow,
                 dt_max=0.05)
    s.extra["qx0"] = qx
    s.extra["qy0"] = qy
    return s
