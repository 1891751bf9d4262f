"""CPU-only checks of the C interface: the library builds, loads and exports
every function include/flood.h declares; host-only entry points behave."""
import ctypes as C
import math
import os
import re

import pytest

import paper_2204_10323_amd as fl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "flood.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fl_[a-z_0-9]+)\s*\(", src)))


def test_header_lists_match_binding():
    assert _declared() == sorted(fl.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = fl.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_default_params_host_only():
    p = fl.default_params()
    assert p.g == 9.81 and p.alpha == 0.7 and p.dt_max == 0.1 and p.h_eps == 1e-4
    assert p.dt_fixed == 0.0 and math.isinf(p.t_end) and p.steps_per_graph == 60
    assert p.positivity == 1


def test_null_context_calls_are_rejected():
    L = fl.lib()
    assert L.fl_init_grid(None, 4, 4, 1.0) == fl.FL_EINVAL
    assert L.fl_step(None, 1) == fl.FL_EINVAL
    assert L.fl_commit(None) == fl.FL_EINVAL
    L.fl_destroy(None)
    assert isinstance(L.fl_last_error(None), bytes)


def test_create_rejects_bad_precision():
    h = C.c_void_p()
    assert fl.lib().fl_create(C.byref(h), 0, None, 7) == fl.FL_EINVAL
    assert b"precision" in fl.lib().fl_last_error(None)
