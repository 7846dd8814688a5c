"""Full approximation scheme driver (Section 3) and dual time stepping
(Section 2, eq. "nonlin-eq"; Section 6: implicit Euler start, then BDF2).

Level numbering here: 0 is the finest level (the paper counts from the
coarsest).  One cycle on level l:

    presmooth nu1 times (one smoothing step on the coarsest level)
    if a coarser level exists:
        r_l = s_l - F_l(u_l)
        u~ = R u_l                       (volume-weighted agglomeration)
        s_{l+1} = F_{l+1}(u~) + R r_l    (eq. "coarse-nonlin-eq")
        cycle(l+1) gamma times           (gamma = 2: the paper's W-cycle)
        u_l += P (u_{l+1} - u~)          (bilinear prolongation)

Readings: on RANS levels the coarse operators keep the viscous flux (the
paper only states that the convective part becomes first-order JST), with
the eddy viscosity of the finer level restricted by volume-weighted
agglomeration whenever the cycle descends, frozen on that level until the
next descent (laminar, mu_t = 0, before the first one); without it the
W-cycle diverges for RANS on boundary-layer grids.  The smoother on a
coarse level drives F_l(u) - s_l to zero (the
printed "s_l - F_l" has the opposite sign of a pseudo-time residual); R of
the per-volume residual is its volume-weighted mean; the bilinear
prolongation weights the parent and its three neighbours on the fine
cell's side by 9/16, 3/16, 3/16, 1/16, takes the partner across a wake cut
and the parent's value where a neighbour does not exist; c* is limited to
20 for the first two cycles of a solve (Section 6); the residual norm is
the RMS of the density component of F over the fine cells.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import gas
from .bc import fill_ghosts
from .geometry import NG, CGRID, build_levels
from .precond import Blocks
from .residual import (baldwin_lomax, local_time_step, padded_eddy_viscosity,
                       split_residual)
from .smoother import SCHEMES, additive_iteration

EULER, RANS = 0, 1


@dataclass
class Params:
    model: int = EULER
    scheme: int = 0                 # smoother.AW3
    eta: float = 0.5
    d_cut: float = 0.5
    cfl: float = 1.0e4
    cfl_ramp: float = 20.0
    n_ramp: int = 2
    ramp_growth: float = 1.0
    n_levels: int = 1
    cycle_gamma: int = 1
    nu1: int = 1
    kappa2c: float = 0.125
    mach: float = 0.8
    alpha_deg: float = 0.0
    reynolds: float = 1.0e7
    prandtl: float = 0.75
    prandtl_t: float = 0.9
    # 0: the printed convective blocks (eqs. "d-l-u-matrices-W" / "-J");
    # 1: plus the thin-layer viscous scalar on RANS levels (extension)
    viscous_blocks: int = 0
    # pseudo time step reading: 0: c* Omega / (r_xi + r_eta);
    # 1: c* Omega / max(r_xi, r_eta)
    dt_form: int = 1


def restrict(lev_f, lev_c, v):
    """Volume-weighted agglomeration of a (4, nj, ni) field."""
    w = v * lev_f.vol
    s = ((w[:, 0::2, 0::2] + w[:, 0::2, 1::2]) + w[:, 1::2, 0::2]) + w[:, 1::2, 1::2]
    return s / lev_c.vol


def restrict_scalar(lev_f, lev_c, m):
    """Volume-weighted agglomeration of a (nj, ni) field."""
    w = m * lev_f.vol
    return (((w[0::2, 0::2] + w[0::2, 1::2]) + w[1::2, 0::2]) + w[1::2, 1::2]) / lev_c.vol


def prolong(lev_f, lev_c, e):
    """Bilinear prolongation of a coarse correction e (4, njc, nic)."""
    nic, njc = lev_c.ni, lev_c.nj
    ii = np.arange(lev_f.ni)
    jj = np.arange(lev_f.nj)
    I = ii // 2
    J = jj // 2
    In = I + np.where(ii % 2 == 0, -1, 1)
    Jn = J + np.where(jj % 2 == 0, -1, 1)
    vi = (In >= 0) & (In < nic)
    vj = (Jn >= 0) & (Jn < njc)
    Inc = np.clip(In, 0, nic - 1)
    Jnc = np.clip(Jn, 0, njc - 1)
    cutc = lev_c.cut_mask()
    JJ, II = np.meshgrid(J, I, indexing="ij")
    JN, IN = np.meshgrid(Jnc, Inc, indexing="ij")
    VI = np.broadcast_to(vi[None, :], JJ.shape)
    VJ = np.broadcast_to(vj[:, None], JJ.shape)
    below = np.broadcast_to((Jn < 0)[:, None], JJ.shape)
    e0 = e[:, JJ, II]
    e1 = np.where(VI, e[:, JJ, IN], e0)
    across2 = below & cutc[II]
    e2 = np.where(VJ, e[:, JN, II],
                  np.where(across2, e[:, np.zeros_like(JJ), nic - 1 - II], e0))
    across3 = below & VI & cutc[IN]
    e3 = np.where(VI & VJ, e[:, JN, IN],
                  np.where(across3, e[:, np.zeros_like(JJ), nic - 1 - IN], e0))
    return (((9.0 * e0 + 3.0 * e1) + 3.0 * e2) + e3) * 0.0625


class Solver:
    """State of one case on all levels, advanced by smoother iterations,
    FAS cycles and physical time steps."""

    def __init__(self, x, y, topology: int, n_wake: int, par: Params, u0):
        self.par = par
        self.levels = build_levels(x, y, topology, n_wake, par.n_levels)
        self.uinf = gas.freestream(par.mach, par.alpha_deg)
        self.U = []
        for lev in self.levels:
            self.U.append(np.zeros((4, lev.nj + 2 * NG, lev.ni + 2 * NG)))
        self.set_u(0, u0)
        L = len(self.levels)
        self.s = [None] * L
        self.un = [None] * L
        self.unm1 = [None] * L
        self.dt = 0.0
        self.bdf = 0
        self.n_cycles = 0
        self.mut = np.zeros((self.levels[0].nj, self.levels[0].ni))
        # padded eddy viscosity of the coarse levels (restricted)
        self.mutc = [None] + [padded_eddy_viscosity(lev, np.zeros((lev.nj, lev.ni)))
                              for lev in self.levels[1:]]
        self.alpha, self.beta, self.aw = SCHEMES[par.scheme]

    # ---------------------------------------------------------------- state
    def u(self, l: int = 0):
        lev = self.levels[l]
        return self.U[l][:, NG:NG + lev.nj, NG:NG + lev.ni].copy()

    def set_u(self, l, u):
        lev = self.levels[l]
        self.U[l][:, NG:NG + lev.nj, NG:NG + lev.ni] = u

    def padded(self, l, u):
        lev = self.levels[l]
        Up = np.zeros((4, lev.nj + 2 * NG, lev.ni + 2 * NG))
        Up[:, NG:NG + lev.nj, NG:NG + lev.ni] = u
        fill_ghosts(Up, lev, self.uinf, noslip=self.par.model == RANS)
        return Up

    # ------------------------------------------------------------ operators
    def tau(self):
        if self.bdf == 2:
            return 3.0 / (2.0 * self.dt)
        if self.bdf == 1:
            return 1.0 / self.dt
        return 0.0

    def time_src(self, l, u):
        if self.bdf == 2:
            return ((3.0 * u - 4.0 * self.un[l]) + self.unm1[l]) / (2.0 * self.dt)
        if self.bdf == 1:
            return (u - self.un[l]) / self.dt
        return None

    def mutp(self, l):
        if self.par.model != RANS:
            return None
        if l == 0:
            return padded_eddy_viscosity(self.levels[0], self.mut)
        return self.mutc[l]

    def split(self, l, u, mutp=None, with_forcing=True):
        Up = self.padded(l, u)
        return split_residual(self.levels[l], Up, self.par, l == 0, mutp,
                              self.time_src(l, u), self.s[l] if with_forcing else None)

    def residual(self, l: int = 0, with_forcing=True, u=None):
        """F_l(u) - s_l (or F_l(u) without the forcing); the eddy
        viscosity is evaluated at u on the fine level."""
        if u is None:
            u = self.u(l)
        mutp = None
        if l == 0 and self.par.model == RANS:
            Up = self.padded(0, u)
            mutp = padded_eddy_viscosity(self.levels[0],
                                         baldwin_lomax(self.levels[0], Up, self.par))
        elif self.par.model == RANS:
            mutp = self.mutc[l]
        Fc, Fv = self.split(l, u, mutp, with_forcing)
        return Fc + Fv

    def cfl_now(self):
        par = self.par
        if self.n_cycles < par.n_ramp:
            return min(par.cfl, par.cfl_ramp)
        if par.ramp_growth > 1.0:
            k = self.n_cycles - par.n_ramp + 1
            # once the ramp has reached c* it stays there (the power is not
            # formed past that point, where it would overflow)
            if par.cfl_ramp <= 0.0 or k * np.log(par.ramp_growth) >= np.log(par.cfl / par.cfl_ramp):
                return par.cfl
            return min(par.cfl, par.cfl_ramp * par.ramp_growth ** k)
        return par.cfl

    # -------------------------------------------------------------- smoother
    def prepare(self, l, cfl=None):
        """Frozen quantities of one smoother iteration at the current state:
        dt*, the eddy viscosity (fine level) and the SGS blocks."""
        lev = self.levels[l]
        u0 = self.u(l)
        Up = self.padded(l, u0)
        dts = local_time_step(lev, Up, self.cfl_now() if cfl is None else cfl, self.par.dt_form)
        mutp = None
        if l == 0 and self.par.model == RANS:
            self.mut = baldwin_lomax(lev, Up, self.par)
            mutp = padded_eddy_viscosity(lev, self.mut)
        elif self.par.model == RANS:
            mutp = self.mutc[l]
        blocks = Blocks(lev, Up, dts, self.par, self.tau(), self.aw,
                        mutp if self.par.viscous_blocks else None)
        return u0, dts, mutp, blocks

    def increment(self, blocks, dts):
        if self.aw:
            return lambda r: blocks.apply(dts * r)
        return lambda r: dts * blocks.apply(r)

    def smooth(self, l: int = 0, cfl=None):
        u0, dts, mutp, blocks = self.prepare(l, cfl)
        split = lambda u: self.split(l, u, mutp)
        u_new = additive_iteration(u0, split, self.increment(blocks, dts),
                                   self.alpha, self.beta)
        self.set_u(l, u_new)

    # ------------------------------------------------------------------ FAS
    # Section 3: level l + 1 (coarser; this module counts from the finest
    # level 0) solves eq. "coarse-nonlin-eq", s_{l+1} - F_{l+1}(u_{l+1}) = 0,
    # whose forcing makes the restricted fine state satisfy it up to the
    # restricted fine residual; the change the coarse solve makes to that
    # restricted state is the fine level's correction.
    def transfer_eddy_viscosity(self, l: int):
        """RANS: the eddy viscosity of level l at its current state (the
        Baldwin-Lomax model on the finest level, the restricted one below),
        restricted to level l + 1 and frozen there for the coarse solve."""
        lev_f, lev_c = self.levels[l], self.levels[l + 1]
        if l == 0:
            m = baldwin_lomax(lev_f, self.padded(0, self.u(0)), self.par)
        else:
            m = self.mutc[l][NG:NG + lev_f.nj, NG:NG + lev_f.ni]
        self.mutc[l + 1] = padded_eddy_viscosity(lev_c, restrict_scalar(lev_f, lev_c, m))

    def coarse_problem(self, l: int):
        """Set up eq. "coarse-nonlin-eq" on level l + 1: its state starts at
        the volume-weighted restriction u~ = R u_l, and its forcing is
        s_{l+1} = F_{l+1}(u~) + R r_l with the defect r_l = s_l - F_l(u_l)
        of level l (s_0 = 0 on the finest level).  Returns u~."""
        lev_f, lev_c = self.levels[l], self.levels[l + 1]
        F = self.residual(l, with_forcing=False)
        defect = -F if self.s[l] is None else self.s[l] - F
        u_restricted = restrict(lev_f, lev_c, self.u(l))
        self.set_u(l + 1, u_restricted)
        self.s[l + 1] = None
        self.s[l + 1] = (self.residual(l + 1, with_forcing=False, u=u_restricted)
                         + restrict(lev_f, lev_c, defect))
        return u_restricted

    def correct(self, l: int, u_restricted):
        """u_l += P (u_{l+1} - u~): the bilinear prolongation of what the
        coarse solve changed."""
        change = self.u(l + 1) - u_restricted
        self.set_u(l, self.u(l) + prolong(self.levels[l], self.levels[l + 1], change))

    def cycle(self, l: int = 0):
        """One FAS cycle from level l: nu1 smoothing steps (one on the
        coarsest level), then, above the coarsest level, the coarse problem,
        cycle_gamma coarse cycles (1: V-cycle, 2: W-cycle) and the
        correction."""
        coarsest = l == len(self.levels) - 1
        for _ in range(1 if coarsest else self.par.nu1):
            self.smooth(l)
        if coarsest:
            return
        if self.par.model == RANS:
            self.transfer_eddy_viscosity(l)
        u_restricted = self.coarse_problem(l)
        for _ in range(self.par.cycle_gamma):
            self.cycle(l + 1)
        self.correct(l, u_restricted)

    def norm(self, F=None):
        if F is None:
            F = self.residual(0)
        return float(np.sqrt(np.sum(F[0] * F[0]) / F[0].size))

    def run_cycles(self, n: int, drop_orders: float = None):
        hist = [self.norm()]
        for _ in range(n):
            self.cycle(0)
            self.n_cycles += 1
            hist.append(self.norm())
            if drop_orders is not None and hist[-1] <= hist[0] * 10.0 ** (-drop_orders):
                break
            if not np.isfinite(hist[-1]):
                break
        return np.array(hist)

    # ------------------------------------------------------ moving mesh
    def set_motion(self, dalpha_deg: float, rate_deg: float, pivot=(0.25, 0.0)):
        """Rigid-body pitching: the body is turned nose-up by dalpha about
        the pivot, i.e. the whole mesh rotates by -dalpha, turning at
        -rate (degrees per unit time); the free stream keeps its angle.
        Reading: moving-mesh (ALE) finite volumes, Section 2 does not state
        the grid-motion terms."""
        from .geometry import rotated
        if not hasattr(self, "levels_ref"):
            self.levels_ref = self.levels
        theta = -dalpha_deg * (np.pi / 180.0)
        omega = -rate_deg * (np.pi / 180.0)
        self.levels = [rotated(lev, theta, omega, pivot[0], pivot[1]) for lev in self.levels_ref]

    # ---------------------------------------------------------- dual time
    def begin_time_step(self, dt: float, alpha_deg: float = None):
        """Shift the time levels and switch to the physical-time equation:
        implicit Euler on the first step, BDF2 afterwards.  A new angle of
        attack turns the free stream at the far field."""
        first = self.un[0] is None
        u = self.u(0)
        self.unm1 = self.un if not first else [None] * len(self.levels)
        self.un = [u]
        for l in range(1, len(self.levels)):
            self.un.append(restrict(self.levels[l - 1], self.levels[l], self.un[l - 1]))
        self.dt = dt
        self.bdf = 1 if first else 2
        self.n_cycles = 0
        if alpha_deg is not None:
            self.par.alpha_deg = alpha_deg
            self.uinf = gas.freestream(self.par.mach, alpha_deg)
