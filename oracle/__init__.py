"""FP64 CPU oracle of the flood step -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is the plain C definition in `flood_oracle.c` (and
the reverse-mode sweep in `flood_oracle_adjoint.c`) behind ctypes, built with
gcc.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "flood_oracle.c"), os.path.join(_HERE, "flood_oracle_adjoint.c")]
_LIB = os.environ.get("FLOOD_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        srcs = [s for s in _SRC if os.path.exists(s)]
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                        "-fopenmp", "-fPIC", "-shared", "-I", _HERE, "-o", tmp, *srcs, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("dx", C.c_double), ("g", C.c_double), ("alpha", C.c_double),
                ("dt_max", C.c_double), ("h_eps", C.c_double), ("dt_fixed", C.c_double),
                ("t_end", C.c_double), ("positivity", C.c_int32),
                ("in_side", C.c_int32), ("in_first", C.c_int32), ("in_count", C.c_int32),
                ("in_slope", C.c_double), ("nsamp", C.c_int32),
                ("ts", C.POINTER(C.c_double)), ("qs", C.POINTER(C.c_double)),
                ("out_side", C.c_int32), ("out_first", C.c_int32), ("out_count", C.c_int32),
                ("out_slope", C.c_double),
                ("friction_vector", C.c_int32), ("boundary_cell_area", C.c_int32)]


class Clock(C.Structure):
    _fields_ = [("t", C.c_double), ("last_dt", C.c_double), ("steps", C.c_int64),
                ("v_in", C.c_double), ("v_out", C.c_double), ("done", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_run.argtypes = [C.POINTER(_Problem), dp, dp, dp, dp, dp, C.POINTER(Clock),
                              C.c_int64, C.c_int32]
        L.orc_run.restype = C.c_int
        L.orc_volume.argtypes = [C.c_int32, C.c_int32, C.c_double, dp]
        L.orc_volume.restype = C.c_double
        L.orc_inflow_split.argtypes = [C.c_int32, dp, dp, C.c_double, C.c_double, dp]
        L.orc_inflow_split.restype = C.c_double
        L.orc_inflow_split_area.argtypes = [C.c_int32, dp, dp, C.c_double, C.c_double, dp]
        L.orc_inflow_split_area.restype = C.c_double
        L.orc_hydrograph.argtypes = [C.c_int32, dp, dp, C.c_double]
        L.orc_hydrograph.restype = C.c_double
        L.orc_face_flux.argtypes = [C.c_double] * 11
        L.orc_face_flux.restype = C.c_double
        L.orc_threads_used.argtypes = [C.c_int32]
        L.orc_threads_used.restype = C.c_int32
        L.orc_adj_run.argtypes = [C.POINTER(_Problem), dp, dp, dp, dp, dp, C.c_int64, C.c_int32,
                                  C.POINTER(C.c_int64), C.c_int32, dp, dp, dp, dp, dp, dp,
                                  C.c_int32]
        L.orc_adj_run.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Run:
    """One oracle simulation: FP64 state promoted from the scenario's float32 inputs.

    Attributes h [ny,nx], qx [ny,nx+1], qy [ny+1,nx] (float64) and `clock`.
    """

    def __init__(self, scen, positivity: bool = True, nthreads: int = 0,
                 n: Optional[np.ndarray] = None, qs: Optional[np.ndarray] = None,
                 friction_vector: bool = False, boundary_cell_area: bool = False):
        self.s = scen
        self.nx, self.ny = scen.nx, scen.ny
        self.z = np.ascontiguousarray(scen.z, dtype=np.float64)
        self.n = np.ascontiguousarray(scen.n if n is None else n, dtype=np.float64)
        self.h = np.ascontiguousarray(scen.h0, dtype=np.float64).copy()
        qx0 = scen.extra.get("qx0")
        qy0 = scen.extra.get("qy0")
        self.qx = (np.zeros((self.ny, self.nx + 1)) if qx0 is None
                   else np.ascontiguousarray(qx0, dtype=np.float64).copy())
        self.qy = (np.zeros((self.ny + 1, self.nx)) if qy0 is None
                   else np.ascontiguousarray(qy0, dtype=np.float64).copy())
        self.nthreads = nthreads
        self.clock = Clock(0.0, 0.0, 0, 0.0, 0.0, 0)
        self.v0 = self.volume()
        p = _Problem()
        p.nx, p.ny, p.dx = scen.nx, scen.ny, scen.dx
        p.g, p.alpha, p.dt_max, p.h_eps = scen.g, scen.alpha, scen.dt_max, scen.h_eps
        p.dt_fixed, p.t_end = scen.dt_fixed, scen.t_end
        p.positivity = 1 if positivity else 0
        p.friction_vector = 1 if friction_vector else 0
        p.boundary_cell_area = 1 if boundary_cell_area else 0
        self._keep = []
        if scen.inflow is not None:
            side, first, count, slope, ts, qsamp = scen.inflow
            ts = np.ascontiguousarray(ts, dtype=np.float64)
            qsamp = np.ascontiguousarray(qsamp if qs is None else qs, dtype=np.float64)
            self._keep += [ts, qsamp]
            p.in_side, p.in_first, p.in_count, p.in_slope = side, first, count, slope
            p.nsamp, p.ts, p.qs = len(ts), _dp(ts), _dp(qsamp)
        else:
            p.in_count = 0
        if scen.outflow is not None:
            side, first, count, slope = scen.outflow
            p.out_side, p.out_first, p.out_count, p.out_slope = side, first, count, slope
        else:
            p.out_count = 0
        self.p = p

    def step(self, nsteps: int) -> int:
        rc = lib().orc_run(C.byref(self.p), _dp(self.z), _dp(self.n), _dp(self.h),
                           _dp(self.qx), _dp(self.qy), C.byref(self.clock), int(nsteps),
                           int(self.nthreads))
        return rc

    def volume(self) -> float:
        return lib().orc_volume(self.nx, self.ny, self.s.dx, _dp(self.h))

    def budget_error(self) -> float:
        """|V - V0 - V_in + V_out| / (V0 + V_in)."""
        v = self.volume()
        c = self.clock
        return abs(v - self.v0 - c.v_in + c.v_out) / max(self.v0 + c.v_in, 1e-300)


def inflow_split(zc, kc, dx: float, Q: float):
    """Eq. (6) solve: returns (W, per-cell face discharge per unit width)."""
    zc = np.ascontiguousarray(zc, dtype=np.float64)
    kc = np.ascontiguousarray(kc, dtype=np.float64)
    q = np.zeros_like(zc)
    W = lib().orc_inflow_split(len(zc), _dp(zc), _dp(kc), dx, Q, _dp(q))
    return W, q


def inflow_split_area(zc, kc, dx: float, Q: float):
    """Eq. (6) with eq. (5) taken literally (A = dx^2): returns (W, per-cell
    face discharge per unit width)."""
    zc = np.ascontiguousarray(zc, dtype=np.float64)
    kc = np.ascontiguousarray(kc, dtype=np.float64)
    q = np.zeros_like(zc)
    W = lib().orc_inflow_split_area(len(zc), _dp(zc), _dp(kc), dx, Q, _dp(q))
    return W, q


def hydrograph(ts, qs, t: float) -> float:
    ts = np.ascontiguousarray(ts, dtype=np.float64)
    qs = np.ascontiguousarray(qs, dtype=np.float64)
    return lib().orc_hydrograph(len(ts), _dp(ts), _dp(qs), t)


def face_flux(hL, hR, zL, zR, nL, nR, q, dx, dt, g=9.81, h_eps=1e-4) -> float:
    return lib().orc_face_flux(hL, hR, zL, zR, nL, nR, q, dx, dt, g, h_eps)


def threads_used(nthreads: int = 0) -> int:
    return lib().orc_threads_used(nthreads)


def adjoint(scen, nsteps: int, gauges, obs_every: int, obs=None, dl_dseries=None,
            n: Optional[np.ndarray] = None, qs: Optional[np.ndarray] = None,
            positivity: bool = True):
    """Reverse-mode gradient of the gauge misfit for a fixed-dt run (FP64).

    gauges: flat cell indices j*nx + i.  Returns (series [nobs, ng], loss,
    grad_n [ny, nx], grad_q [nsamples]).  Either obs (squared misfit) or
    dl_dseries (adjoint seeds) must be given.
    """
    r = Run(scen, positivity=positivity, n=n, qs=qs)
    g = np.ascontiguousarray(gauges, dtype=np.int64)
    nobs = nsteps // obs_every
    series = np.zeros((nobs, len(g)))
    grad_n = np.zeros((scen.ny, scen.nx))
    nsamp = r.p.nsamp if scen.inflow is not None else 0
    grad_q = np.zeros(max(nsamp, 1))
    loss = C.c_double(0.0)
    ob = None if obs is None else np.ascontiguousarray(obs, dtype=np.float64)
    dl = None if dl_dseries is None else np.ascontiguousarray(dl_dseries, dtype=np.float64)
    rc = lib().orc_adj_run(C.byref(r.p), _dp(r.z), _dp(r.n), _dp(r.h), _dp(r.qx), _dp(r.qy),
                           int(nsteps), len(g), g.ctypes.data_as(C.POINTER(C.c_int64)),
                           int(obs_every), None if ob is None else _dp(ob),
                           None if dl is None else _dp(dl), _dp(series), C.byref(loss),
                           _dp(grad_n), _dp(grad_q), 1)
    if rc != 0:
        raise RuntimeError(f"orc_adj_run failed ({rc})")
    return series, loss.value, grad_n, grad_q[:nsamp]
