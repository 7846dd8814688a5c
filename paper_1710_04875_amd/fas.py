"""ctypes binding of the HIP library (include/fas.h).

Argument marshalling only: every step of the solver runs in the library's
kernels.  Device arrays are torch tensors on the current HIP device
(float64, [4][nj][ni]); work is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfas.so")

FAS_OK, FAS_EINVAL, FAS_ENOMEM, FAS_EDEVICE, FAS_DIVERGED, FAS_STALLED, FAS_NOT_CONVERGED = 0, -1, -2, -3, -4, -5, -6
FAS_BOX, FAS_CGRID = 0, 1
FAS_EULER, FAS_RANS_BL = 0, 1
FAS_AW3, FAS_PARK3J, FAS_AW5J, FAS_AW51, FAS_AW52, FAS_PARK51 = range(6)
PARAMS_VERSION = 4

_lib = None


class FasError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("fas status %d: %s" % (status, msg))
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [
        ("version", ctypes.c_int32), ("model", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("n_ramp", ctypes.c_int32),
        ("eta", ctypes.c_double), ("d_cut", ctypes.c_double), ("cfl", ctypes.c_double),
        ("cfl_ramp", ctypes.c_double), ("ramp_growth", ctypes.c_double), ("kappa2c", ctypes.c_double),
        ("mach", ctypes.c_double), ("alpha_deg", ctypes.c_double), ("reynolds", ctypes.c_double),
        ("prandtl", ctypes.c_double), ("prandtl_t", ctypes.c_double),
        ("n_levels", ctypes.c_int32), ("cycle_gamma", ctypes.c_int32), ("nu1", ctypes.c_int32),
        ("precond_fp32", ctypes.c_int32), ("viscous_blocks", ctypes.c_int32), ("dt_form", ctypes.c_int32),
        ("stall_window", ctypes.c_int32), ("stall_orders", ctypes.c_double), ("growth_limit", ctypes.c_double),
        ("adjoint_levels", ctypes.c_int32),
        ("freeze_mut", ctypes.c_int32),
    ]


@dataclass
class Params:
    """Mirror of fas_params (defaults: AW3, robust mode)."""
    model: int = FAS_EULER
    scheme: int = FAS_AW3
    n_ramp: int = 2
    eta: float = 0.5
    d_cut: float = 0.5
    cfl: float = 1.0e4
    cfl_ramp: float = 20.0
    ramp_growth: float = 1.0
    kappa2c: float = 0.125
    mach: float = 0.8
    alpha_deg: float = 0.0
    reynolds: float = 1.0e7
    prandtl: float = 0.75
    prandtl_t: float = 0.9
    n_levels: int = 1
    cycle_gamma: int = 1
    nu1: int = 1
    precond_fp32: int = 0
    viscous_blocks: int = 0
    dt_form: int = 1
    stall_window: int = 0
    stall_orders: float = 0.0
    growth_limit: float = 1.0e8
    adjoint_levels: int = 0
    freeze_mut: int = 0

    def c(self) -> _Params:
        p = _Params()
        p.version = PARAMS_VERSION
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p


EXPORTS = [
    "fas_params_default", "fas_grid_create", "fas_grid_destroy", "fas_grid_set_nodes", "fas_state_create",
    "fas_state_destroy", "fas_state_set_params", "fas_set_state", "fas_get_state", "fas_get_time_levels",
    "fas_get_level", "fas_handoff_pending", "fas_residual", "fas_smooth", "fas_sgs_apply", "fas_cycle",
    "fas_dual_time_step", "fas_profile", "fas_profile_read", "fas_batch_create",
    "fas_batch_destroy", "fas_batch_solve", "fas_batch_sweep_config", "fas_batch_set_sweep_config",
    "fas_sweep_config_count", "fas_sweep_config_info", "fas_batch_profile",
    "fas_batch_profile_read", "fas_forces", "fas_vjp", "fas_param_partials",
    "fas_sgs_apply_transpose", "fas_adjoint_solve", "fas_lift_gradient", "fas_vjp_nodes",
    "fas_lift_gradient_nodes", "fas_set_motion", "fas_dfa", "fas_dfa_noalloc", "fas_vjp_smooth",
    "fas_unsteady_lift_gradient",
    "fas_set_four_lane_limit",
    "fas_last_error",
]
PROF_CLASSES = ("sweep", "residual", "blocks")


def load(path: str = LIB_PATH):
    """Load libfas.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("HIP library %s not built; run python -m paper_1710_04875_amd.build" % path)
    lib = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    i32, f64 = ctypes.c_int32, ctypes.c_double
    sig = {
        "fas_params_default": (None, [ctypes.POINTER(_Params)]),
        "fas_grid_create": (i32, [i32, i32, i32, i32, dp, dp, i32, ctypes.POINTER(vp)]),
        "fas_grid_set_nodes": (i32, [vp, dp, dp]),
        "fas_grid_destroy": (None, [vp]),
        "fas_state_create": (i32, [vp, ctypes.POINTER(_Params), vp, vp, ctypes.POINTER(vp)]),
        "fas_state_destroy": (None, [vp]),
        "fas_state_set_params": (i32, [vp, ctypes.POINTER(_Params)]),
        "fas_set_state": (i32, [vp, vp, vp, vp, f64, f64, i32, i32]),
        "fas_get_time_levels": (i32, [vp, vp, vp, dp, dp, ip, ip]),
        "fas_vjp_smooth": (i32, [vp, vp, vp]),
        "fas_unsteady_lift_gradient": (i32, [vp, i32, f64, dp, i32, f64, i32, i32, f64, dp, dp, dp, ip, dp, ip]),
        "fas_set_four_lane_limit": (ctypes.c_int64, [ctypes.c_int64]),
        "fas_get_state": (i32, [vp, vp, vp]),
        "fas_get_level": (i32, [vp, i32, vp, vp]),
        "fas_handoff_pending": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int64)]),
        "fas_residual": (i32, [vp, i32, vp]),
        "fas_smooth": (i32, [vp, i32, i32]),
        "fas_sgs_apply": (i32, [vp, i32, vp, vp]),
        "fas_cycle": (i32, [vp, i32, f64, dp, ip]),
        "fas_dual_time_step": (i32, [vp, f64, f64, i32, f64, dp, ip]),
        "fas_profile": (i32, [vp, i32]),
        "fas_profile_read": (i32, [vp, dp, ctypes.POINTER(ctypes.c_int64)]),
        "fas_batch_create": (i32, [i32, ctypes.POINTER(vp), vp, i32, i32, ctypes.POINTER(vp)]),
        "fas_batch_destroy": (None, [vp]),
        "fas_batch_solve": (i32, [vp, i32, f64, i32, ip, ip, dp]),
        "fas_batch_sweep_config": (i32, [vp, i32, ip, ip]),
        "fas_batch_set_sweep_config": (i32, [vp, i32, i32]),
        "fas_sweep_config_count": (i32, []),
        "fas_sweep_config_info": (i32, [i32, ip, ip, ip, ip, ip]),
        "fas_batch_profile": (i32, [vp, i32]),
        "fas_batch_profile_read": (i32, [vp, dp, ctypes.POINTER(ctypes.c_int64)]),
        "fas_forces": (i32, [vp, dp, dp, vp]),
        "fas_vjp": (i32, [vp, vp, vp]),
        "fas_param_partials": (i32, [vp, vp, vp, dp]),
        "fas_sgs_apply_transpose": (i32, [vp, vp, vp]),
        "fas_adjoint_solve": (i32, [vp, vp, vp, i32, f64, dp, ip]),
        "fas_lift_gradient": (i32, [vp, i32, f64, dp, dp, dp, ip]),
        "fas_vjp_nodes": (i32, [vp, vp, vp, vp]),
        "fas_lift_gradient_nodes": (i32, [vp, i32, f64, dp, dp, vp, vp, dp, ip]),
        "fas_set_motion": (i32, [vp, f64, f64, f64, f64]),
        "fas_dfa": (i32, [ctypes.POINTER(_DfaCase), i32, vp, vp, vp, vp]),
        "fas_dfa_noalloc": (i32, [ctypes.POINTER(_DfaCase), i32, vp, vp, vp, vp]),
        "fas_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st, allow=()):
    if st != FAS_OK and st not in allow:
        raise FasError(st, _lib.fas_last_error().decode())
    return st


def _dptr(t):
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Grid:
    """Structured grid with its agglomerated levels (host node arrays)."""

    def __init__(self, topology, x, y, n_wake=0, n_levels=1):
        lib = load()
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        self.nj, self.ni = x.shape[0] - 1, x.shape[1] - 1
        self.topology, self.n_wake, self.n_levels = topology, n_wake, n_levels
        h = ctypes.c_void_p()
        _check(lib.fas_grid_create(topology, self.ni, self.nj, n_wake,
                                   x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   n_levels, ctypes.byref(h)))
        self.h = h
        self.x, self.y = x.copy(), y.copy()

    def set_nodes(self, x, y):
        """Move the nodes (same shape): every level's metrics are recomputed;
        states on this grid use them from their next call."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        if x.shape != (self.nj + 1, self.ni + 1) or y.shape != x.shape:
            raise ValueError("node arrays must be (nj + 1, ni + 1)")
        _check(_lib.fas_grid_set_nodes(self.h, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       y.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self.x, self.y = x.copy(), y.copy()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fas_grid_destroy(self.h)
            self.h = None


class State:
    """One flow case on a Grid; every call enqueues on torch's current stream."""

    def __init__(self, grid: Grid, params: Params, u0):
        import torch
        lib = load()
        self.grid = grid
        self.params = params
        self.device = u0.device
        u0 = u0.to(torch.float64).contiguous()
        h = ctypes.c_void_p()
        self._pc = params.c()
        _check(lib.fas_state_create(grid.h, ctypes.byref(self._pc), _dptr(u0), _stream(), ctypes.byref(h)))
        self.h = h
        self._keep = u0

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fas_state_destroy(self.h)
            self.h = None

    def shape(self, level=0):
        return (4, self.grid.nj >> level, self.grid.ni >> level)

    def set_params(self, params: Params):
        self.params = params
        self._pc = params.c()
        _check(_lib.fas_state_set_params(self.h, ctypes.byref(self._pc)))

    def set_state(self, u, un=None, unm1=None, t=0.0, dt=0.0, step=0, n_cycles=0):
        """Restore a checkpoint: the solution, the time levels of the BDF
        step in progress (step >= 1: un; step >= 2: unm1), the clock and the
        cycle count of the current solve (step 0: a steady state)."""
        keep = [u.to(torch_dtype()).contiguous()]
        for v in (un, unm1):
            keep.append(None if v is None else v.to(torch_dtype()).contiguous())
        _check(_lib.fas_set_state(self.h, _dptr(keep[0]), _dptr(keep[1]) if keep[1] is not None else None,
                                  _dptr(keep[2]) if keep[2] is not None else None, float(t), float(dt),
                                  int(step), int(n_cycles)))
        self._keep = keep

    def get_time_levels(self):
        """(un, unm1, t, dt, step, n_cycles); un / unm1 are None when the
        state does not hold them."""
        import torch
        t, dt = ctypes.c_double(0.0), ctypes.c_double(0.0)
        step, nc = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib.fas_get_time_levels(self.h, None, None, ctypes.byref(t), ctypes.byref(dt),
                                        ctypes.byref(step), ctypes.byref(nc)))
        un = torch.empty(self.shape(), dtype=torch.float64, device=self.device) if step.value > 0 else None
        unm1 = torch.empty(self.shape(), dtype=torch.float64, device=self.device) if step.value > 1 else None
        _check(_lib.fas_get_time_levels(self.h, _dptr(un) if un is not None else None,
                                        _dptr(unm1) if unm1 is not None else None, None, None, None, None))
        return un, unm1, t.value, dt.value, step.value, nc.value

    def checkpoint(self):
        """Everything fas_set_state needs to resume this state bitwise."""
        un, unm1, t, dt, step, nc = self.get_time_levels()
        return dict(u=self.get_state(), un=un, unm1=unm1, t=t, dt=dt, step=step, n_cycles=nc)

    def get_state(self, with_mut=False):
        import torch
        u = torch.empty(self.shape(), dtype=torch.float64, device=self.device)
        mut = torch.empty(self.shape()[1:], dtype=torch.float64, device=self.device) if with_mut else None
        _check(_lib.fas_get_state(self.h, _dptr(u), _dptr(mut) if with_mut else None))
        return (u, mut) if with_mut else u

    def get_level(self, level):
        import torch
        u = torch.empty(self.shape(level), dtype=torch.float64, device=self.device)
        s = torch.empty(self.shape(level), dtype=torch.float64, device=self.device)
        _check(_lib.fas_get_level(self.h, level, _dptr(u), _dptr(s)))
        return u, s

    def handoff_pending(self, level=0):
        """Words of a level's band hand-off array not holding the sentinel
        (0 whenever no sweep is running)."""
        n = ctypes.c_int64(0)
        _check(_lib.fas_handoff_pending(self.h, level, ctypes.byref(n)))
        return int(n.value)

    def residual(self, level=0):
        import torch
        F = torch.empty(self.shape(level), dtype=torch.float64, device=self.device)
        _check(_lib.fas_residual(self.h, level, _dptr(F)))
        return F

    def smooth(self, level=0, n_iter=1):
        _check(_lib.fas_smooth(self.h, level, n_iter))

    def sgs_apply(self, r, level=0):
        import torch
        r = r.to(torch.float64).contiguous()
        x = torch.empty_like(r)
        _check(_lib.fas_sgs_apply(self.h, level, _dptr(r), _dptr(x)))
        return x

    def cycle(self, max_cycles, drop_orders=0.0):
        hist = np.zeros(max_cycles + 1)
        n = ctypes.c_int32(0)
        st = _check(_lib.fas_cycle(self.h, max_cycles, drop_orders,
                                   hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(n)),
                    allow=(FAS_NOT_CONVERGED, FAS_DIVERGED, FAS_STALLED))
        return hist[:n.value + 1], st

    def profile(self, enable=True):
        _check(_lib.fas_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        ms = np.zeros(len(PROF_CLASSES))
        n = np.zeros(len(PROF_CLASSES), dtype=np.int64)
        _check(_lib.fas_profile_read(self.h, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return {c: (float(ms[k]), int(n[k])) for k, c in enumerate(PROF_CLASSES)}

    def set_motion(self, dalpha_deg, rate_deg, pivot=(0.25, 0.0)):
        """Rigid-body pitching on a moving mesh: the body turned nose-up by
        dalpha_deg about the pivot, turning at rate_deg per unit time."""
        _check(_lib.fas_set_motion(self.h, dalpha_deg, rate_deg, pivot[0], pivot[1]))

    # ------------------------------------------------------------ adjoint
    def forces(self, with_grad=False):
        """(C_L, C_D[, dC_L/du]) of the wall pressure force."""
        import torch
        cl, cd = ctypes.c_double(0.0), ctypes.c_double(0.0)
        g = torch.empty(self.shape(), dtype=torch.float64, device=self.device) if with_grad else None
        _check(_lib.fas_forces(self.h, ctypes.byref(cl), ctypes.byref(cd), _dptr(g) if with_grad else None))
        return (cl.value, cd.value, g) if with_grad else (cl.value, cd.value)

    def vjp(self, lam):
        """(dF/du)^T lam at the current state (frozen eddy viscosity)."""
        import torch
        lam = lam.to(torch.float64).contiguous()
        out = torch.empty_like(lam)
        _check(_lib.fas_vjp(self.h, _dptr(lam), _dptr(out)))
        return out

    def vjp_smooth(self, lam):
        """(dS/du)^T lam for one fine-level smoother iteration S at frozen
        dt*, blocks and eddy viscosity (the state is left unchanged)."""
        import torch
        lam = lam.to(torch.float64).contiguous()
        out = torch.empty_like(lam)
        _check(_lib.fas_vjp_smooth(self.h, _dptr(lam), _dptr(out)))
        return out

    def param_partials(self):
        """(dF/dalpha_deg, dF/dM, [dC_L/dalpha_deg, dC_L/dM] at fixed u)."""
        import torch
        da = torch.empty(self.shape(), dtype=torch.float64, device=self.device)
        dm = torch.empty_like(da)
        c = np.zeros(2)
        _check(_lib.fas_param_partials(self.h, _dptr(da), _dptr(dm),
                                       c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return da, dm, c

    def sgs_apply_transpose(self, r):
        import torch
        r = r.to(torch.float64).contiguous()
        x = torch.empty_like(r)
        _check(_lib.fas_sgs_apply_transpose(self.h, _dptr(r), _dptr(x)))
        return x

    def adjoint_solve(self, rhs, max_iter, drop_orders, lam0=None):
        import torch
        rhs = rhs.to(torch.float64).contiguous()
        lam = torch.zeros_like(rhs) if lam0 is None else lam0.to(torch.float64).clone().contiguous()
        hist = np.zeros(max_iter + 1)
        n = ctypes.c_int32(0)
        st = _check(_lib.fas_adjoint_solve(self.h, _dptr(rhs), _dptr(lam), max_iter, drop_orders,
                                           hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           ctypes.byref(n)), allow=(FAS_NOT_CONVERGED,))
        return lam, hist[:n.value + 1], st

    def lift_gradient(self, max_iter=2000, drop_orders=10.0):
        """(C_L, [dC_L/dalpha_deg, dC_L/dM], adjoint history, status)."""
        cl = ctypes.c_double(0.0)
        g = np.zeros(2)
        hist = np.zeros(max_iter + 1)
        n = ctypes.c_int32(0)
        st = _check(_lib.fas_lift_gradient(self.h, max_iter, drop_orders, ctypes.byref(cl),
                                           g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           ctypes.byref(n)), allow=(FAS_NOT_CONVERGED,))
        return cl.value, g, hist[:n.value + 1], st

    def vjp_nodes(self, lam):
        """((dF/dx)^T lam, (dF/dy)^T lam) on the node arrays (nj + 1, ni + 1)
        at the current state (frozen eddy viscosity)."""
        import torch
        lam = lam.to(torch.float64).contiguous()
        dx = torch.empty((self.grid.nj + 1, self.grid.ni + 1), dtype=torch.float64, device=self.device)
        dy = torch.empty_like(dx)
        _check(_lib.fas_vjp_nodes(self.h, _dptr(lam), _dptr(dx), _dptr(dy)))
        return dx, dy

    def lift_gradient_nodes(self, max_iter=2000, drop_orders=10.0):
        """(C_L, [dC_L/dalpha_deg, dC_L/dM], dC_L/dx, dC_L/dy (node arrays),
        adjoint history, status) at a converged state."""
        import torch
        cl = ctypes.c_double(0.0)
        g = np.zeros(2)
        dx = torch.empty((self.grid.nj + 1, self.grid.ni + 1), dtype=torch.float64, device=self.device)
        dy = torch.empty_like(dx)
        hist = np.zeros(max_iter + 1)
        n = ctypes.c_int32(0)
        st = _check(_lib.fas_lift_gradient_nodes(self.h, max_iter, drop_orders, ctypes.byref(cl),
                                                 g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 _dptr(dx), _dptr(dy),
                                                 hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 ctypes.byref(n)), allow=(FAS_NOT_CONVERGED,))
        return cl.value, g, dx, dy, hist[:n.value + 1], st

    def unsteady_lift_gradient(self, dt, alpha_deg, max_inner=200, inner_drop=11.0, checkpoint_every=1,
                               adj_max_iter=2000, adj_drop=10.0):
        """Time-averaged lift J of len(alpha_deg) - 1 dual time steps from this
        (converged, steady) state and its gradient by the checkpointed
        unsteady adjoint: (J, dJ/dM, dJ/dalpha_n per degree (n = 0..N),
        adjoint iterations per step, adjoint orders reached per step,
        recomputed steps)."""
        a = np.ascontiguousarray(alpha_deg, dtype=np.float64)
        n = len(a) - 1
        J, dm = ctypes.c_double(0.0), ctypes.c_double(0.0)
        da = np.zeros(n + 1)
        its = np.zeros(n + 1, dtype=np.int32)
        orders = np.zeros(n + 1)
        rec = ctypes.c_int32(0)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(_lib.fas_unsteady_lift_gradient(self.h, n, dt, a.ctypes.data_as(dp), max_inner, inner_drop,
                                               checkpoint_every, adj_max_iter, adj_drop, ctypes.byref(J),
                                               ctypes.byref(dm), da.ctypes.data_as(dp),
                                               its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                               orders.ctypes.data_as(dp), ctypes.byref(rec)))
        return J.value, dm.value, da, its, orders, rec.value

    def dual_time_step(self, dt, alpha_deg, max_inner, drop_orders):
        hist = np.zeros(max_inner + 1)
        n = ctypes.c_int32(0)
        st = _check(_lib.fas_dual_time_step(self.h, dt, alpha_deg, max_inner, drop_orders,
                                            hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            ctypes.byref(n)),
                    allow=(FAS_NOT_CONVERGED, FAS_DIVERGED, FAS_STALLED))
        return hist[:n.value + 1], st


def set_four_lane_limit(max_cells):
    """Launch-size rule of the residual and block kernels (cells per launch
    up to which the four-lane variants run; < 0: default).  Returns the
    previous value."""
    return int(load().fas_set_four_lane_limit(int(max_cells)))


def torch_dtype():
    import torch
    return torch.float64


SWEEP_FOUR_THREADS, SWEEP_ONE_THREAD, SWEEP_BANDED, SWEEP_EIGHT_THREADS, SWEEP_EIGHT_BANDED = 0, 1, 2, 3, 4


class _DfaCase(ctypes.Structure):
    _fields_ = [("u", ctypes.c_double * 4), ("scheme", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("unsteady", ctypes.c_int32), ("cstar", ctypes.c_double),
                ("d", ctypes.c_double), ("eta", ctypes.c_double), ("ar", ctypes.c_double),
                ("c", ctypes.c_double), ("precond", ctypes.c_int32), ("unsplit", ctypes.c_int32),
                ("mesh", ctypes.c_int32), ("reserved", ctypes.c_int32)]


DFA_SGS, DFA_EXACT, DFA_NONE = 0, 1, 2
DFA_MESH_AR_DX, DFA_MESH_DX_OVER_AR = 0, 1


@dataclass
class DfaCase:
    """Mirror of fas_dfa_case: one Fourier analysis of a smoother (the
    linearisation state at Mach 0.8, alpha 0 by default; ny defaults to
    nx * ar)."""
    u: tuple = (1.0, 1.0, 0.0, 3.290)
    scheme: int = FAS_AW3
    cstar: float = 3.0
    d: float = 0.5
    eta: float = 0.8
    ar: float = 1.0
    c: float = 200.0
    nx: int = 8
    ny: int = 0
    unsteady: int = 1
    precond: int = 0
    unsplit: int = 0
    mesh: int = 0

    def c_struct(self) -> _DfaCase:
        x = _DfaCase()
        for k in range(4):
            x.u[k] = float(self.u[k])
        x.scheme, x.nx = int(self.scheme), int(self.nx)
        x.ny = int(self.ny) if self.ny else int(round(self.nx * self.ar))
        x.unsteady = int(self.unsteady)
        x.cstar, x.d, x.eta, x.ar, x.c = float(self.cstar), float(self.d), float(self.eta), float(self.ar), float(self.c)
        x.precond, x.unsplit, x.mesh, x.reserved = int(self.precond), int(self.unsplit), int(self.mesh), 0
        return x


def dfa(cases, with_radius=False):
    """Amplification and smoothing factors (float64 tensors on the current
    device, one per case) and, on request, the spectral radius of every pair
    of phase angles (cases concatenated, Theta_x slowest)."""
    import torch
    lib = load()
    arr = (_DfaCase * len(cases))(*[c.c_struct() for c in cases])
    dev = torch.device("cuda", torch.cuda.current_device())
    amp = torch.empty(len(cases), dtype=torch.float64, device=dev)
    smooth = torch.empty_like(amp)
    total = sum(int(a.nx) * int(a.ny) for a in arr)
    rad = torch.empty(total, dtype=torch.float64, device=dev) if with_radius else None
    _check(lib.fas_dfa(arr, len(cases), ctypes.c_void_p(amp.data_ptr()), ctypes.c_void_p(smooth.data_ptr()),
                       ctypes.c_void_p(rad.data_ptr() if rad is not None else 0),
                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return (amp, smooth, rad) if with_radius else (amp, smooth)


def sweep_config_count():
    """Number of sweep configurations (indices for Batch.set_sweep_config)."""
    return int(load().fas_sweep_config_count())


def sweep_config_info(cfg):
    """(kind, threads, rows per workgroup, FP64 depth, FP32 depth) of a sweep
    configuration; kind is SWEEP_FOUR_THREADS, SWEEP_ONE_THREAD,
    SWEEP_BANDED (row bands of four-thread rows), SWEEP_EIGHT_THREADS or
    SWEEP_EIGHT_BANDED (row bands of eight-thread rows)."""
    v = [ctypes.c_int32(0) for _ in range(5)]
    _check(load().fas_sweep_config_info(cfg, *[ctypes.byref(x) for x in v]))
    return tuple(int(x.value) for x in v)


class Batch:
    """Independent steady cases advanced together (one launch per kernel
    over all cases, optionally replayed from a captured HIP graph).  The
    batch works in place on the states' buffers; keep them alive.  groups > 1
    runs that many case groups concurrently, each on its own stream."""

    def __init__(self, states, autotune=True, groups=1):
        lib = load()
        self.states = list(states)
        arr = (ctypes.c_void_p * len(self.states))(*[st.h.value for st in self.states])
        h = ctypes.c_void_p()
        _check(lib.fas_batch_create(len(self.states), arr, _stream(), 1 if autotune else 0, int(groups),
                                    ctypes.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fas_batch_destroy(self.h)
            self.h = None

    def solve(self, max_cycles, drop_orders=0.0, use_graph=True):
        """Returns (per-case histories, per-case status, worst status)."""
        n = len(self.states)
        hist = np.zeros((n, max_cycles + 1))
        nd = np.zeros(n, dtype=np.int32)
        stv = np.zeros(n, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int32)
        st = _check(_lib.fas_batch_solve(self.h, max_cycles, drop_orders, 1 if use_graph else 0,
                                         nd.ctypes.data_as(ip), stv.ctypes.data_as(ip),
                                         hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    allow=(FAS_NOT_CONVERGED, FAS_DIVERGED, FAS_STALLED))
        return [hist[c, :nd[c] + 1].copy() for c in range(n)], stv, st

    def sweep_config(self, level):
        c, r = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib.fas_batch_sweep_config(self.h, level, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    def set_sweep_config(self, level, cfg):
        _check(_lib.fas_batch_set_sweep_config(self.h, level, cfg))

    def profile(self, enable=True):
        _check(_lib.fas_batch_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        ms = np.zeros(len(PROF_CLASSES))
        n = np.zeros(len(PROF_CLASSES), dtype=np.int64)
        _check(_lib.fas_batch_profile_read(self.h, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return {c: (float(ms[k]), int(n[k])) for k, c in enumerate(PROF_CLASSES)}


def _steady_lift_fn():
    import torch

    class SteadyLift(torch.autograd.Function):
        """C_L(M, alpha_deg[, x_nodes, y_nodes]) of the converged steady
        solution on a State: the forward pass sets the flow parameters (and
        moves the grid's nodes if given) and runs FAS cycles to the drop,
        the backward pass solves the adjoint for dC_L/d(M, alpha) and, if
        the nodes are inputs, dC_L/d(x, y) of every node."""

        @staticmethod
        def forward(ctx, mach, alpha_deg, x_nodes, y_nodes, state, max_cycles, drop_orders, adj_iter, adj_drop,
                    allow_unconverged):
            p = state.params
            p.mach = float(mach)
            p.alpha_deg = float(alpha_deg)
            state.set_params(p)
            ctx.nodes = x_nodes is not None or y_nodes is not None
            if ctx.nodes:
                g = state.grid
                x = x_nodes.detach().cpu().numpy() if x_nodes is not None else g.x
                y = y_nodes.detach().cpu().numpy() if y_nodes is not None else g.y
                g.set_nodes(x, y)
            _, st = state.cycle(max_cycles, drop_orders)
            if st != FAS_OK and not allow_unconverged:
                raise FasError(st, "steady_lift: the primal solve did not reach the requested drop "
                                   "(pass allow_unconverged=True to accept it)")
            cl, _ = state.forces()
            ctx.state = state
            ctx.adj = (adj_iter, adj_drop)
            ctx.allow = allow_unconverged
            ctx.node_meta = [(t.device, t.dtype) if t is not None else None for t in (x_nodes, y_nodes)]
            return torch.tensor(cl, dtype=torch.float64)

        @staticmethod
        def backward(ctx, g):
            gx = gy = None
            if ctx.nodes:
                _, grad, dx, dy, _, st = ctx.state.lift_gradient_nodes(*ctx.adj)
                mx, my = ctx.node_meta
                if mx is not None:
                    gx = g.to(dx.device) * dx
                    gx = gx.to(device=mx[0], dtype=mx[1])
                if my is not None:
                    gy = g.to(dy.device) * dy
                    gy = gy.to(device=my[0], dtype=my[1])
            else:
                _, grad, _, st = ctx.state.lift_gradient(*ctx.adj)
            if st != FAS_OK and not ctx.allow:
                raise FasError(st, "steady_lift: the adjoint solve did not reach the requested drop "
                                   "(pass allow_unconverged=True to accept it)")
            return (g * grad[1], g * grad[0], gx, gy, None, None, None, None, None, None)

    return SteadyLift


def steady_lift(mach, alpha_deg, state, max_cycles=400, drop_orders=10.0, adj_iter=2000, adj_drop=10.0,
                x_nodes=None, y_nodes=None, allow_unconverged=False):
    """Differentiable C_L(M, alpha) (torch scalars) of a converged State; with
    x_nodes / y_nodes ((nj + 1, ni + 1) tensors) also differentiable in the
    grid-node coordinates (the forward pass moves the State's grid there).
    Raises FasError when the primal (forward) or the adjoint (backward) does
    not reach its drop, unless allow_unconverged.  For RANS the gradient is
    that of the frozen-turbulence adjoint: the Baldwin-Lomax eddy viscosity
    is held at the converged state, so its own sensitivity is left out."""
    return _steady_lift_fn().apply(mach, alpha_deg, x_nodes, y_nodes, state, max_cycles, drop_orders, adj_iter,
                                   adj_drop, allow_unconverged)
