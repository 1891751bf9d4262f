"""Argument checks of the Python binding that need no GPU: arrays read by the
library are converted to the context's element type and checked against the
shape the call describes; arrays the library writes in place must already
have that type, shape and layout (a converted copy would hide the result)."""
import numpy as np
import pytest

import paper_2204_10323_amd as fl


def test_inputs_are_converted_and_shape_checked():
    a = np.arange(12, dtype=np.float64).reshape(3, 4)
    p, stride, dev, keep = fl._as_input(a, np.float32, (3, 4), "z")
    assert dev == 0 and stride == 4 and keep.dtype == np.float32
    assert np.array_equal(keep, a.astype(np.float32))
    strided = np.zeros((3, 8), np.float32)[:, ::2]
    p, stride, dev, keep = fl._as_input(strided, np.float32, (3, 4), "z", packed=True)
    assert stride == 4 and keep.flags.c_contiguous
    with pytest.raises(ValueError, match="shape"):
        fl._as_input(a, np.float32, (4, 3), "z")


def test_outputs_must_match_exactly():
    ok = np.zeros((3, 4), np.float32)
    p, stride, dev = fl._as_output(ok, np.float32, (3, 4), "out")
    assert stride == 4 and dev == 0 and p.value == ok.ctypes.data
    wide = np.zeros((3, 6), np.float32)[:, :4]        # rows contiguous, row stride 6
    p, stride, dev = fl._as_output(wide, np.float32, (3, 4), "out")
    assert stride == 6
    with pytest.raises(ValueError, match="contiguous"):
        fl._as_output(wide, np.float32, (3, 4), "out", packed=True)
    with pytest.raises(ValueError):
        fl._as_output(np.zeros((3, 4), np.float64), np.float32, (3, 4), "out")
    with pytest.raises(ValueError, match="shape"):
        fl._as_output(np.zeros((4, 3), np.float32), np.float32, (3, 4), "out")
    with pytest.raises(ValueError, match="contiguous"):
        fl._as_output(np.zeros((4, 3), np.float32).T, np.float32, (3, 4), "out")
    with pytest.raises(ValueError):
        fl._as_output([[0.0] * 4] * 3, np.float32, (3, 4), "out")


def test_torch_host_tensors():
    torch = pytest.importorskip("torch")
    t = torch.arange(12, dtype=torch.float64).reshape(3, 4)
    p, stride, dev, keep = fl._as_input(t, np.float32, (3, 4), "z")
    assert dev == 0 and keep.dtype == np.float32
    o = torch.zeros((3, 4), dtype=torch.float32)
    p, stride, dev = fl._as_output(o, np.float32, (3, 4), "out")
    assert dev == 0 and p.value == o.data_ptr()
    with pytest.raises(ValueError):
        fl._as_output(torch.zeros((3, 4), dtype=torch.float64), np.float32, (3, 4), "out")


def test_discharge_sweep_argument_checks():
    """The sweep helper refuses bad settings before it creates a context."""
    import numpy as np
    import pytest
    from paper_2204_10323_amd.sweep import discharge_sweep
    z = np.zeros((8, 8), np.float32)
    n = np.full((8, 8), 0.03, np.float32)
    sec = (0, 2, 3, 1e-3)
    with pytest.raises(ValueError):
        discharge_sweep(z, n, 1.0, sec, None, [1.0], 10, 0.1, mode="fast")
    with pytest.raises(ValueError):
        discharge_sweep(z, n, 1.0, sec, None, [1.0], 0, 0.1)
    with pytest.raises(ValueError):
        discharge_sweep(z, n, 1.0, sec, None, [1.0], 10, 0.1, steps_per_entry=4)
    with pytest.raises(ValueError):
        discharge_sweep(z, n, 1.0, sec, None, [1.0], 10, 0.1, steps_per_entry=3, active_tiles=True)
