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
    # the printed convective blocks, the directional pseudo time step, no
    # stall test, divergence beyond a 1e8 growth
    assert (p.viscous_blocks, p.dt_form, p.stall_window, p.growth_limit) == (0, 1, 0, 1.0e8)
    assert p.adjoint_levels == 0             # adjoint preconditioner over every level
    assert p.freeze_mut == 0                 # eddy viscosity follows the state
    assert ctypes.sizeof(fas._Params) == 160
    # the binding's defaults are the library's
    dflt = fas.Params()
    for name, _ in fas._Params._fields_:
        if name != "version":
            assert getattr(dflt, name) == getattr(p, name), name


def test_four_lane_limit_setting():
    from paper_1710_04875_amd import fas
    old = fas.set_four_lane_limit(0)
    try:
        assert old == 65536
        assert fas.set_four_lane_limit(-1) == 0
        assert fas.set_four_lane_limit(123) == 65536
    finally:
        fas.set_four_lane_limit(-1)


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
    assert lib.fas_batch_create(0, None, None, 0, 1, ctypes.byref(h)) == fas.FAS_EINVAL
    assert lib.fas_batch_solve(None, 1, 0.0, 0, None, None, None) == fas.FAS_EINVAL
    assert lib.fas_cycle(None, 1, 0.0, None, None) == fas.FAS_EINVAL
    assert lib.fas_residual(None, 0, None) == fas.FAS_EINVAL
    assert lib.fas_set_state(None, None, None, None, 0.0, 0.0, 0, 0) == fas.FAS_EINVAL
    assert lib.fas_get_time_levels(None, None, None, None, None, None, None) == fas.FAS_EINVAL
    assert lib.fas_vjp_smooth(None, None, None) == fas.FAS_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    from paper_1710_04875_amd import fas
    saved = fas._lib
    fas._lib = None
    try:
        with pytest.raises(ImportError):
            fas.load(str(tmp_path / "absent.so"))
    finally:
        fas._lib = saved
