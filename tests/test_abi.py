"""The C ABI without a GPU: the library loads, exports every function that
include/fas.h declares, and rejects bad arguments before touching a
device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fas.h")
LIB = os.path.join(ROOT, "paper_1710_04875_amd", "libfas.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfas.so not built")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fas_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_function_is_exported():
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_every_declared_function():
    from paper_1710_04875_amd import fas
    assert sorted(fas.EXPORTS) == declared()


def test_params_layout_and_defaults():
    from paper_1710_04875_amd import fas
    lib = fas.load()
    p = fas._Params()
    lib.fas_params_default(ctypes.byref(p))
    assert p.version == fas.PARAMS_VERSION
    assert p.scheme == fas.FAS_AW3 and p.model == fas.FAS_EULER
    # robust mode of the paper: eta 0.5, d 0.5, c* 1e4 after 2 cycles at 20
    assert (p.eta, p.d_cut, p.cfl, p.cfl_ramp, p.n_ramp) == (0.5, 0.5, 1.0e4, 20.0, 2)
    assert ctypes.sizeof(fas._Params) == 120


def test_argument_errors_without_device():
    from paper_1710_04875_amd import fas
    lib = fas.load()
    x = np.zeros((9, 9))
    dp = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    # bad topology, bad level count, indivisible sizes, too tall, bad wake
    assert lib.fas_grid_create(7, 8, 8, 0, dp, dp, 1, ctypes.byref(h)) == fas.FAS_EINVAL
    assert lib.fas_grid_create(0, 8, 8, 0, dp, dp, 0, ctypes.byref(h)) == fas.FAS_EINVAL
    assert lib.fas_grid_create(0, 10, 8, 0, dp, dp, 3, ctypes.byref(h)) == fas.FAS_EINVAL
    assert lib.fas_grid_create(0, 8, 1024, 0, dp, dp, 1, ctypes.byref(h)) == fas.FAS_EINVAL
    assert lib.fas_grid_create(1, 8, 8, 4, dp, dp, 1, ctypes.byref(h)) == fas.FAS_EINVAL
    assert b"n_wake" in lib.fas_last_error()
    assert lib.fas_grid_create(0, 8, 8, 0, None, dp, 1, ctypes.byref(h)) == fas.FAS_EINVAL
    assert lib.fas_state_create(None, None, None, None, ctypes.byref(h)) == fas.FAS_EINVAL
    assert lib.fas_batch_create(0, None, None, 0, ctypes.byref(h)) == fas.FAS_EINVAL
    assert lib.fas_batch_solve(None, 1, 0.0, 0, None, None, None) == fas.FAS_EINVAL
    assert lib.fas_cycle(None, 1, 0.0, None, None) == fas.FAS_EINVAL
    assert lib.fas_residual(None, 0, None) == fas.FAS_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    from paper_1710_04875_amd import fas
    saved = fas._lib
    fas._lib = None
    try:
        with pytest.raises(ImportError):
            fas.load(str(tmp_path / "absent.so"))
    finally:
        fas._lib = saved
