"""Python binding of libflood (include/flood.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libflood.so; this module
only converts arrays and calls the C functions of the same names.  Importing
works without a GPU; loading the library raises if it has not been built.
"""
from __future__ import annotations

import atexit
import ctypes as C
import math
import os
import weakref
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FLOOD_LIB") or os.path.join(_HERE, "libflood.so")

FL_OK, FL_EINVAL, FL_ENOMEM, FL_EHIP, FL_ESTATE, FL_ENONFINITE = range(6)
FL_F32, FL_F64 = 0, 1
FL_WEST, FL_EAST, FL_SOUTH, FL_NORTH = range(4)
FL_FRICTION_FACE, FL_FRICTION_VECTOR = 0, 1
FL_BOUNDARY_SECTION, FL_BOUNDARY_CELL_AREA = 0, 1
FL_NOALLOC_MAX_MEMBERS = 256   # members fl_batch_run_noalloc's device scratch holds
STATUS_NAMES = {0: "FL_OK", 1: "FL_EINVAL", 2: "FL_ENOMEM", 3: "FL_EHIP", 4: "FL_ESTATE",
                5: "FL_ENONFINITE"}

# Every symbol include/flood.h declares.
EXPORTS = [
    "fl_default_params", "fl_create", "fl_init_grid", "fl_set_dem", "fl_set_manning",
    "fl_set_inflow", "fl_set_outflow", "fl_set_params", "fl_set_state", "fl_commit", "fl_step",
    "fl_advance", "fl_get_depth", "fl_get_discharge", "fl_get_report", "fl_last_error",
    "fl_destroy", "fl_time_steps", "fl_set_tiling", "fl_device_bytes",
    "fl_batch_create", "fl_batch_set_tiling", "fl_batch_autotune", "fl_batch_run",
    "fl_batch_time", "fl_batch_last_error", "fl_batch_destroy",
    "fl_adj_setup", "fl_adj_forward", "fl_adj_backward", "fl_autotune", "fl_set_fusion",
    "fl_workspace_bytes", "fl_bind_workspace", "fl_get_state", "fl_autotune_fusion",
    "fl_set_active_tiles", "fl_active_items", "fl_set_variant", "fl_batch_run_noalloc",
    "fl_batch_set_fusion",
]


class FloodError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class fl_params(C.Structure):
    _fields_ = [("g", C.c_double), ("alpha", C.c_double), ("dt_max", C.c_double),
                ("h_eps", C.c_double), ("dt_fixed", C.c_double), ("t_end", C.c_double),
                ("steps_per_graph", C.c_int32), ("positivity", C.c_int32)]


class fl_report(C.Structure):
    _fields_ = [("t", C.c_double), ("last_dt", C.c_double), ("steps", C.c_int64),
                ("v0", C.c_double), ("v_in", C.c_double), ("v_out", C.c_double),
                ("v_now", C.c_double), ("done", C.c_int32), ("nonfinite", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}

    def budget_error(self) -> float:
        return abs(self.v_now - self.v0 - self.v_in + self.v_out) / max(self.v0 + self.v_in, 1e-300)


_lib = None

# Open contexts and batches.  At interpreter exit they are closed by an atexit
# hook, batches first (they borrow their members), while the HIP runtime is
# still up; after that no finalizer makes a HIP call (objects collected during
# interpreter shutdown are left to the process exit).
_open_ctxs: "weakref.WeakSet" = weakref.WeakSet()
_open_batches: "weakref.WeakSet" = weakref.WeakSet()
_exiting = False


@atexit.register
def _close_all():
    global _exiting
    try:
        for b in list(_open_batches):
            b.close()
        for f in list(_open_ctxs):
            f.close()
    finally:
        _exiting = True


def lib() -> C.CDLL:
    """The loaded libflood.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        # PyTorch ships its own HIP runtime (soname libamdhip64.so.7, linked by
        # torch as libamdhip64.so).  Load it first so that libflood binds to
        # that same runtime instead of mapping a second one from /opt/rocm:
        # two HIP/HSA runtimes in one process cannot share the device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "fl_default_params": (None, [C.POINTER(fl_params)]),
            "fl_create": (C.c_int, [C.POINTER(vp), C.c_int, vp, C.c_int]),
            "fl_init_grid": (C.c_int, [vp, i32, i32, dbl]),
            "fl_set_dem": (C.c_int, [vp, vp, i64, C.c_int]),
            "fl_set_manning": (C.c_int, [vp, vp, i64, C.c_int]),
            "fl_set_inflow": (C.c_int, [vp, C.c_int, i32, i32, dbl, C.POINTER(dbl),
                                        C.POINTER(dbl), i32]),
            "fl_set_outflow": (C.c_int, [vp, C.c_int, i32, i32, dbl]),
            "fl_set_params": (C.c_int, [vp, C.POINTER(fl_params)]),
            "fl_set_state": (C.c_int, [vp, vp, vp, vp, dbl, C.c_int]),
            "fl_commit": (C.c_int, [vp]),
            "fl_step": (C.c_int, [vp, i64]),
            "fl_advance": (C.c_int, [vp, dbl]),
            "fl_get_depth": (C.c_int, [vp, vp, i64, C.c_int]),
            "fl_get_discharge": (C.c_int, [vp, vp, vp, C.c_int]),
            "fl_get_report": (C.c_int, [vp, C.POINTER(fl_report)]),
            "fl_last_error": (C.c_char_p, [vp]),
            "fl_destroy": (None, [vp]),
            "fl_time_steps": (C.c_int, [vp, i64, C.POINTER(dbl)]),
            "fl_set_tiling": (C.c_int, [vp, i32, i32]),
            "fl_device_bytes": (C.c_size_t, [vp]),
            "fl_batch_create": (C.c_int, [C.POINTER(vp), i32, C.POINTER(vp)]),
            "fl_batch_set_tiling": (C.c_int, [vp, i32, i32]),
            "fl_batch_autotune": (C.c_int, [vp, C.POINTER(i32), i32, i32, C.POINTER(i32),
                                            C.POINTER(dbl)]),
            "fl_batch_run": (C.c_int, [vp, i64]),
            "fl_batch_run_noalloc": (C.c_int, [vp, i64]),
            "fl_batch_set_fusion": (C.c_int, [vp, i32, i32, i32]),
            "fl_batch_time": (C.c_int, [vp, i64, C.POINTER(dbl)]),
            "fl_batch_last_error": (C.c_char_p, [vp]),
            "fl_batch_destroy": (None, [vp]),
            "fl_adj_setup": (C.c_int, [vp, C.POINTER(i32), i32, i32, vp, i64, C.c_int, i32]),
            "fl_adj_forward": (C.c_int, [vp, i64, vp, C.c_int, C.POINTER(dbl)]),
            "fl_adj_backward": (C.c_int, [vp, vp, C.POINTER(dbl), C.c_int, C.POINTER(dbl)]),
            "fl_autotune": (C.c_int, [vp, C.POINTER(i32), i32, i32, C.POINTER(i32), C.POINTER(dbl)]),
            "fl_set_fusion": (C.c_int, [vp, i32, i32, i32]),
            "fl_workspace_bytes": (C.c_size_t, [i32, i32, C.c_int, C.c_uint32]),
            "fl_bind_workspace": (C.c_int, [vp, vp, C.c_size_t]),
            "fl_get_state": (C.c_int, [vp, vp, vp, vp, C.POINTER(dbl), C.c_int]),
            "fl_autotune_fusion": (C.c_int, [vp, i32, C.POINTER(i32), C.POINTER(dbl)]),
            "fl_set_active_tiles": (C.c_int, [vp, i32]),
            "fl_set_variant": (C.c_int, [vp, i32, i32]),
            "fl_active_items": (C.c_int, [vp, C.POINTER(i64), C.POINTER(i64)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(ctx, status: int):
    if status != FL_OK:
        msg = lib().fl_last_error(ctx)
        raise FloodError(status, msg.decode() if msg else "")


def default_params(**over) -> fl_params:
    p = fl_params()
    lib().fl_default_params(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def _np_dtype(prec: int):
    return np.float64 if prec == FL_F64 else np.float32


def _torch_stream_ptr():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def _check_shape(a, shape, name):
    if shape is not None and tuple(a.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(a.shape)}, expected {tuple(shape)}")


def _as_input(a, dtype, shape=None, name="array", packed=False):
    """(pointer, row_stride, on_device, keepalive) for a 2-D numpy array or
    torch tensor read by the library: converted to the element type (a copy
    if needed), checked against `shape`, rows contiguous, and with `packed`
    the row stride equal to the row length (calls that take no stride)."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            _check_shape(a, shape, name)
            tdt = torch.float64 if dtype == np.float64 else torch.float32
            if a.is_cuda:
                t = a.detach().to(tdt)
                if (packed and not t.is_contiguous()) or t.stride(-1) != 1:
                    t = t.contiguous()
                return C.c_void_p(t.data_ptr()), t.stride(0) if t.dim() > 1 else t.numel(), 1, t
            a = a.detach().cpu().numpy()
    except ImportError:
        pass
    arr = np.ascontiguousarray(a, dtype=dtype)
    _check_shape(arr, shape, name)
    return C.c_void_p(arr.ctypes.data), arr.shape[-1] if arr.ndim > 1 else arr.size, 0, arr


def _as_output(a, dtype, shape, name, packed=False):
    """(pointer, row_stride, on_device) of an array the library writes in
    place: it must already have the element type and shape, rows contiguous,
    and with `packed` no gaps between rows (no copy is made, so a mismatch
    is an error rather than a result written into a temporary)."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            _check_shape(a, shape, name)
            tdt = torch.float64 if dtype == np.float64 else torch.float32
            if a.dtype != tdt:
                raise ValueError(f"{name}: dtype {a.dtype}, expected {tdt}")
            if a.stride(-1) != 1 or (packed and not a.is_contiguous()):
                raise ValueError(f"{name}: must be contiguous")
            stride = a.stride(0) if a.dim() > 1 else a.numel()
            if a.is_cuda:
                return C.c_void_p(a.data_ptr()), stride, 1
            return C.c_void_p(a.data_ptr()), stride, 0
    except ImportError:
        pass
    if not isinstance(a, np.ndarray) or a.dtype != np.dtype(dtype):
        raise ValueError(f"{name}: a numpy array of {np.dtype(dtype)} (or a tensor) is needed")
    _check_shape(a, shape, name)
    if a.strides[-1] != a.itemsize or (packed and not a.flags.c_contiguous):
        raise ValueError(f"{name}: must be contiguous")
    stride = a.strides[0] // a.itemsize if a.ndim > 1 else a.size
    return C.c_void_p(a.ctypes.data), stride, 0


class Flood:
    """One flood context (fl_ctx): a grid, its inputs, and its device state.

    Methods map one-to-one onto the C functions fl_<name>; arrays may be numpy
    (host) or torch CUDA tensors (device).
    """

    def __init__(self, nx: int, ny: int, dx: float, precision: str = "f32", device: int = 0,
                 stream=None):
        self.prec = FL_F64 if precision in ("f64", "fp64", "double") else FL_F32
        self.dtype = _np_dtype(self.prec)
        self.nx, self.ny, self.dx = int(nx), int(ny), float(dx)
        h = C.c_void_p()
        s = stream if stream is not None else _torch_stream_ptr()
        st = lib().fl_create(C.byref(h), device, s, self.prec)
        if st != FL_OK:
            raise FloodError(st, lib().fl_last_error(None).decode())
        self.ctx = h
        _open_ctxs.add(self)
        _check(self.ctx, lib().fl_init_grid(self.ctx, self.nx, self.ny, self.dx))

    # -- inputs
    def set_dem(self, z):
        p, stride, dev, keep = _as_input(z, self.dtype, (self.ny, self.nx), "z")
        _check(self.ctx, lib().fl_set_dem(self.ctx, p, stride, dev))

    def set_manning(self, n):
        p, stride, dev, keep = _as_input(n, self.dtype, (self.ny, self.nx), "n")
        _check(self.ctx, lib().fl_set_manning(self.ctx, p, stride, dev))

    def set_inflow(self, side: int, first: int, count: int, slope: float, t_s, q_m3s):
        ts = np.ascontiguousarray(t_s, dtype=np.float64)
        qs = np.ascontiguousarray(q_m3s, dtype=np.float64)
        dp = C.POINTER(C.c_double)
        _check(self.ctx, lib().fl_set_inflow(self.ctx, side, first, count, slope,
                                             ts.ctypes.data_as(dp), qs.ctypes.data_as(dp),
                                             len(ts)))

    def set_outflow(self, side: int, first: int, count: int, slope: float):
        _check(self.ctx, lib().fl_set_outflow(self.ctx, side, first, count, slope))

    def set_params(self, **kw):
        p = default_params(**kw)
        _check(self.ctx, lib().fl_set_params(self.ctx, C.byref(p)))

    def set_state(self, h, qx=None, qy=None, t: float = 0.0):
        """Initial state (fl_set_state): h [ny, nx], qx [ny, nx+1] and qy
        [ny+1, nx] (None: zero), all in host memory or all on the device."""
        ph, _, dev, k1 = _as_input(h, self.dtype, (self.ny, self.nx), "h", packed=True)
        px = py = None
        k2 = k3 = None
        if qx is not None:
            px, _, d2, k2 = _as_input(qx, self.dtype, (self.ny, self.nx + 1), "qx", packed=True)
            if d2 != dev:
                raise ValueError("set_state: h and qx must both be host or both device arrays")
        if qy is not None:
            py, _, d3, k3 = _as_input(qy, self.dtype, (self.ny + 1, self.nx), "qy", packed=True)
            if d3 != dev:
                raise ValueError("set_state: h and qy must both be host or both device arrays")
        _check(self.ctx, lib().fl_set_state(self.ctx, ph, px, py, float(t), dev))

    def set_tiling(self, cells_per_lane: int = 0, rows_per_item: int = 0):
        _check(self.ctx, lib().fl_set_tiling(self.ctx, cells_per_lane, rows_per_item))

    def _side_length(self, side: int) -> int:
        return self.ny if side in (FL_WEST, FL_EAST) else self.nx

    def set_inflow_fraction(self, side: int, f_start: float, f_end: float, slope: float, t_s, q_m3s):
        """set_inflow on the section given as fractions of the side (fraction_section)."""
        first, count = fraction_section(self._side_length(side), f_start, f_end)
        self.set_inflow(side, first, count, slope, t_s, q_m3s)

    def set_outflow_fraction(self, side: int, f_start: float, f_end: float, slope: float):
        """set_outflow on the section given as fractions of the side (fraction_section)."""
        first, count = fraction_section(self._side_length(side), f_start, f_end)
        self.set_outflow(side, first, count, slope)

    def set_fusion(self, steps_per_launch: int, cells_per_lane: int = 0, rows_per_item: int = 0):
        """Steps per launch (1, 2 or 3) and the multi-step kernel's tiling (fl_set_fusion)."""
        _check(self.ctx, lib().fl_set_fusion(self.ctx, steps_per_launch, cells_per_lane,
                                             rows_per_item))

    def set_variant(self, friction: str = "face", boundary: str = "section"):
        """Method variant (fl_set_variant): friction "face" (default) or "vector";
        boundary "section" (default) or "cell_area"."""
        fr = {"face": FL_FRICTION_FACE, "vector": FL_FRICTION_VECTOR}.get(friction)
        bd = {"section": FL_BOUNDARY_SECTION, "cell_area": FL_BOUNDARY_CELL_AREA}.get(boundary)
        if fr is None or bd is None:
            raise ValueError("set_variant: friction 'face'|'vector', boundary 'section'|'cell_area'")
        _check(self.ctx, lib().fl_set_variant(self.ctx, fr, bd))

    def set_active_tiles(self, on=True):
        """Active-tile (wet-region) skipping (fl_set_active_tiles): False/0 off,
        True/1 the per-item skip test, 2 single-step launches select a list of
        items first."""
        mode = 2 if on == 2 else (1 if on else 0)
        _check(self.ctx, lib().fl_set_active_tiles(self.ctx, mode))

    def active_items(self):
        """(work items the next step computes, work items per step) (fl_active_items)."""
        nxt, tot = C.c_int64(), C.c_int64()
        _check(self.ctx, lib().fl_active_items(self.ctx, C.byref(nxt), C.byref(tot)))
        return nxt.value, tot.value

    def commit(self):
        _check(self.ctx, lib().fl_commit(self.ctx))

    def autotune(self, candidates, trial_steps: int = 10):
        """Pick the fastest (cells_per_lane, rows_per_item) by frozen trial steps (fl_autotune)."""
        flat = [int(v) for pair in candidates for v in pair]
        arr = (C.c_int32 * len(flat))(*flat)
        best = (C.c_int32 * 2)()
        ms = C.c_double()
        _check(self.ctx, lib().fl_autotune(self.ctx, arr, len(candidates), trial_steps, best,
                                           C.byref(ms)))
        return (best[0], best[1]), ms.value

    def autotune_fusion(self, trial_steps: int = 20):
        """Keep one step or the committed k steps per launch, whichever frozen trials find faster
        (fl_autotune_fusion); needs a commit after set_fusion(2 or 3)."""
        spl = C.c_int32()
        ms = C.c_double()
        _check(self.ctx, lib().fl_autotune_fusion(self.ctx, int(trial_steps), C.byref(spl),
                                                  C.byref(ms)))
        return spl.value, ms.value

    # -- stepping
    def step(self, nsteps: int):
        _check(self.ctx, lib().fl_step(self.ctx, int(nsteps)))

    def advance(self, seconds: float):
        _check(self.ctx, lib().fl_advance(self.ctx, float(seconds)))

    def time_steps(self, nsteps: int) -> float:
        ms = C.c_double()
        _check(self.ctx, lib().fl_time_steps(self.ctx, int(nsteps), C.byref(ms)))
        return ms.value

    # -- outputs
    def get_depth(self, out=None) -> np.ndarray:
        if out is not None:
            p, stride, dev = _as_output(out, self.dtype, (self.ny, self.nx), "out")
            _check(self.ctx, lib().fl_get_depth(self.ctx, p, stride, dev))
            return out
        h = np.empty((self.ny, self.nx), dtype=self.dtype)
        _check(self.ctx, lib().fl_get_depth(self.ctx, C.c_void_p(h.ctypes.data), self.nx, 0))
        return h

    def get_discharge(self) -> Tuple[np.ndarray, np.ndarray]:
        qx = np.empty((self.ny, self.nx + 1), dtype=self.dtype)
        qy = np.empty((self.ny + 1, self.nx), dtype=self.dtype)
        _check(self.ctx, lib().fl_get_discharge(self.ctx, C.c_void_p(qx.ctypes.data),
                                                C.c_void_p(qy.ctypes.data), 0))
        return qx, qy

    def get_state(self):
        """(h, qx, qy, t) in the layout set_state takes (fl_get_state)."""
        h = np.empty((self.ny, self.nx), dtype=self.dtype)
        qx = np.empty((self.ny, self.nx + 1), dtype=self.dtype)
        qy = np.empty((self.ny + 1, self.nx), dtype=self.dtype)
        t = C.c_double()
        _check(self.ctx, lib().fl_get_state(self.ctx, C.c_void_p(h.ctypes.data),
                                            C.c_void_p(qx.ctypes.data),
                                            C.c_void_p(qy.ctypes.data), C.byref(t), 0))
        return h, qx, qy, t.value

    def workspace_bytes(self, two_step: bool = False, active_tiles: bool = False) -> int:
        flags = (1 if two_step else 0) | (2 if active_tiles else 0)
        return int(lib().fl_workspace_bytes(self.nx, self.ny, self.prec, flags))

    def bind_workspace(self, buf):
        """Carve the commit buffers from a caller-owned device tensor (kept
        referenced here); None unbinds (fl_bind_workspace)."""
        if buf is None:
            _check(self.ctx, lib().fl_bind_workspace(self.ctx, None, 0))
            self._ws = None
            return
        if not getattr(buf, "is_cuda", False) or not buf.is_contiguous():
            raise ValueError("bind_workspace: a contiguous device tensor is needed")
        nbytes = buf.numel() * buf.element_size()
        _check(self.ctx, lib().fl_bind_workspace(self.ctx, C.c_void_p(buf.data_ptr()), nbytes))
        self._ws = buf

    def get_report(self, check: bool = True) -> fl_report:
        r = fl_report()
        st = lib().fl_get_report(self.ctx, C.byref(r))
        if check:
            _check(self.ctx, st)
        return r

    # -- reverse mode
    def adj_setup(self, gauges, obs_every: int, obs=None, ckpt_stride: int = 0):
        g = np.ascontiguousarray(gauges, dtype=np.int32)
        self._nsamp = None
        if obs is None:
            st = lib().fl_adj_setup(self.ctx, g.ctypes.data_as(C.POINTER(C.c_int32)), len(g),
                                    obs_every, None, 0, 0, ckpt_stride)
        else:
            nobs = obs.shape[0]
            p, _, dev, keep = _as_input(obs, self.dtype, (nobs, len(g)), "obs", packed=True)
            st = lib().fl_adj_setup(self.ctx, g.ctypes.data_as(C.POINTER(C.c_int32)), len(g),
                                    obs_every, p, nobs, dev, ckpt_stride)
        _check(self.ctx, st)
        self._ngauges, self._obs_every = len(g), obs_every

    def adj_forward(self, nsteps: int, out=None):
        """Run nsteps keeping checkpoints; returns (series, loss)."""
        loss = C.c_double()
        nobs = nsteps // self._obs_every
        self._nobs = nobs
        if out is not None:
            p, _, dev = _as_output(out, self.dtype, (nobs, self._ngauges), "out", packed=True)
            _check(self.ctx, lib().fl_adj_forward(self.ctx, int(nsteps), p, dev, C.byref(loss)))
            return out, loss.value
        series = np.empty((nobs, self._ngauges), dtype=self.dtype)
        _check(self.ctx, lib().fl_adj_forward(self.ctx, int(nsteps), C.c_void_p(series.ctypes.data),
                                               0, C.byref(loss)))
        return series, loss.value

    def adj_backward(self, dl_dseries=None, nsamples: int = 0, grad_n_out=None):
        """Gradients (grad_n [ny, nx] float64, grad_q [nsamples] float64) of the last adj_forward."""
        dp = C.POINTER(C.c_double)
        gq = np.zeros(max(1, nsamples), dtype=np.float64)
        pdl = None
        keep = None
        if dl_dseries is not None:
            shape = (getattr(self, "_nobs", dl_dseries.shape[0]), self._ngauges)
            pdl, _, _, keep = _as_input(dl_dseries, self.dtype, shape, "dl_dseries", packed=True)
        if grad_n_out is not None:
            pg, _, gdev = _as_output(grad_n_out, np.float64, (self.ny, self.nx), "grad_n_out",
                                     packed=True)
            _check(self.ctx, lib().fl_adj_backward(self.ctx, pdl, C.cast(pg, dp), gdev,
                                                   gq.ctypes.data_as(dp)))
            return grad_n_out, gq[:nsamples]
        gn = np.zeros((self.ny, self.nx), dtype=np.float64)
        _check(self.ctx, lib().fl_adj_backward(self.ctx, pdl, gn.ctypes.data_as(dp), 0,
                                               gq.ctypes.data_as(dp)))
        return gn, gq[:nsamples]

    def device_bytes(self) -> int:
        return int(lib().fl_device_bytes(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            lib().fl_destroy(self.ctx)
            self.ctx = None
        _open_ctxs.discard(self)

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batched ensemble (fl_batch) of committed Flood contexts stepped by one launch."""

    def __init__(self, members):
        self.members = list(members)
        arr = (C.c_void_p * len(self.members))(*[m.ctx for m in self.members])
        h = C.c_void_p()
        st = lib().fl_batch_create(C.byref(h), len(self.members), arr)
        if st != FL_OK:
            raise FloodError(st, lib().fl_batch_last_error(None).decode())
        self.b = h
        _open_batches.add(self)

    def _check(self, st):
        if st != FL_OK:
            raise FloodError(st, lib().fl_batch_last_error(self.b).decode())

    def _live(self):
        # the C batch borrows its members: a closed member must not be stepped
        if not getattr(self, "b", None):
            raise ValueError("the batch is closed")
        if any(m.ctx is None for m in self.members):
            raise ValueError("a member of the batch was closed")

    def set_tiling(self, cells_per_lane: int, rows_per_item: int):
        self._live()
        self._check(lib().fl_batch_set_tiling(self.b, cells_per_lane, rows_per_item))

    def set_fusion(self, steps_per_entry: int, cells_per_lane: int = 0, rows_per_item: int = 0):
        """fl_batch_set_fusion: one, two or three steps per queue entry (more
        than one needs members committed with fusion 2 or 3 and without active
        tiles)."""
        self._live()
        self._check(lib().fl_batch_set_fusion(self.b, steps_per_entry, cells_per_lane, rows_per_item))

    def autotune(self, candidates, trial_steps: int = 20):
        self._live()
        flat = [int(v) for pair in candidates for v in pair]
        arr = (C.c_int32 * len(flat))(*flat)
        best = (C.c_int32 * 2)()
        ms = C.c_double()
        self._check(lib().fl_batch_autotune(self.b, arr, len(candidates), trial_steps, best,
                                            C.byref(ms)))
        return (best[0], best[1]), ms.value

    def run(self, nsteps: int):
        self._live()
        self._check(lib().fl_batch_run(self.b, int(nsteps)))

    def run_noalloc(self, nsteps: int):
        """fl_batch_run_noalloc: the same steps with the library's static device
        scratch (no allocation during the call)."""
        self._live()
        self._check(lib().fl_batch_run_noalloc(self.b, int(nsteps)))

    def time(self, nsteps: int) -> float:
        self._live()
        ms = C.c_double()
        self._check(lib().fl_batch_time(self.b, int(nsteps), C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "b", None):
            lib().fl_batch_destroy(self.b)
            self.b = None
        _open_batches.discard(self)

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


def fraction_section(length: int, f_start: float, f_end: float):
    """(first, count) of the cells along a side of `length` cells whose centre
    lies at a fraction (k + 1/2) / length of the side within [f_start, f_end]:
    the paper's way of placing a boundary section (its fraction_start and
    fraction_end of a side, Methods).  (0, 0) when no centre lies inside."""
    if length < 1:
        raise ValueError("fraction_section: length must be >= 1")
    k = np.arange(length)
    c = (k + 0.5) / length
    sel = np.nonzero((c >= f_start) & (c <= f_end))[0]
    if sel.size == 0:
        return 0, 0
    return int(sel[0]), int(sel.size)


def from_scenario(sc, precision: str = "f32", device: int = 0, stream=None, commit: bool = True,
                  cells_per_lane: int = 0, rows_per_item: int = 0, fusion=None,
                  active_tiles: bool = False, variant=None, **param_over) -> Flood:
    """A committed context for a synthetic scenario (see the `synth` module)."""
    f = Flood(sc.nx, sc.ny, sc.dx, precision, device, stream)
    f.set_dem(sc.z)
    f.set_manning(sc.n)
    if sc.inflow is not None:
        side, first, count, slope, ts, qs = sc.inflow
        f.set_inflow(side, first, count, slope, ts, qs)
    if sc.outflow is not None:
        f.set_outflow(*sc.outflow)
    params = dict(g=sc.g, alpha=sc.alpha, dt_max=sc.dt_max, h_eps=sc.h_eps,
                  dt_fixed=sc.dt_fixed, t_end=sc.t_end)
    params.update(param_over)
    f.set_params(**params)
    qx0, qy0 = sc.extra.get("qx0"), sc.extra.get("qy0")
    if qx0 is not None or qy0 is not None or np.any(sc.h0):
        f.set_state(sc.h0, qx0, qy0, 0.0)
    if cells_per_lane or rows_per_item:
        f.set_tiling(cells_per_lane, rows_per_item)
    if fusion is not None:
        f.set_fusion(*((fusion,) if isinstance(fusion, int) else tuple(fusion)))
    if active_tiles:
        f.set_active_tiles(active_tiles)
    if variant is not None:
        f.set_variant(*variant)
    if commit:
        f.commit()
    return f
