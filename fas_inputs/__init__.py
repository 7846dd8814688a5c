"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only builds input data: grid node coordinates and initial
conservative states.  It holds none of the solver's arithmetic (no fluxes,
no residuals, no preconditioner, no multigrid), so that the two
implementations it feeds stay independent.

Stand-ins for the paper's meshes (Section 6: NACA 64A010 and RAE 2822
C-meshes, which are not available): an algebraic C-grid around a symmetric
10 %-thick NACA 4-digit section with a boundary-layer-stretched inner half
of the j-lines, and a jittered Cartesian box for the Euler case.

Array conventions
-----------------
* nodes: ``x[J, I]``, ``y[J, I]`` with ``I = 0..ni`` fastest, ``J = 0..nj``.
* cell states: ``u[k, j, i]`` (k = rho, rho*u, rho*v, rho*E), float64.
* Grids are right-handed (i, j) so that cell areas are positive.
* C-grid: i runs from the lower wake outflow, along the lower wake, around
  the airfoil (lower surface trailing edge -> leading edge -> upper surface)
  and out along the upper wake; j runs from the wall / wake cut outward.
  Wake nodes coincide pairwise: node (I, 0) == node (ni - I, 0) for
  I <= n_wake.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4

BOX = 0
CGRID = 1


# --------------------------------------------------------------------------
# small 1-D distribution helpers
# --------------------------------------------------------------------------
def _geometric_ratio(n: int, first: float, total: float) -> float:
    """Ratio r > 1 with first*(r^n - 1)/(r - 1) == total (bisection)."""
    if first * n >= total:
        raise ValueError("first spacing too large for a stretched distribution")
    lo, hi = 1.0 + 1e-12, 2.0
    while first * (hi ** n - 1.0) / (hi - 1.0) < total:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s = first * (mid ** n - 1.0) / (mid - 1.0)
        if s < total:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _geometric_spacing(n: int, first: float, total: float) -> np.ndarray:
    r = _geometric_ratio(n, first, total)
    d = first * r ** np.arange(n)
    d *= total / d.sum()
    return d


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------
def box_grid(ni: int = 64, nj: int = 64, ratio: float = 1.1,
             jitter: float = 0.05, seed: int = 1):
    """Jittered unit box, x uniform, y geometric from the wall side y=0.

    Interior nodes are moved by U(-jitter, jitter) times the smaller of the
    two adjacent spacings in each direction; boundary nodes stay on the box.
    """
    xs = np.linspace(0.0, 1.0, ni + 1)
    dy = ratio ** np.arange(nj)
    ys = np.concatenate([[0.0], np.cumsum(dy)])
    ys /= ys[-1]
    x, y = np.meshgrid(xs, ys)                      # [J, I]
    rng = np.random.default_rng(seed)
    jx = rng.uniform(-jitter, jitter, size=(nj - 1, ni - 1))
    jy = rng.uniform(-jitter, jitter, size=(nj - 1, ni - 1))
    dxl = np.minimum(np.diff(xs)[:-1], np.diff(xs)[1:])        # per interior I
    dyl = np.minimum(np.diff(ys)[:-1], np.diff(ys)[1:])        # per interior J
    x = x.copy()
    y = y.copy()
    x[1:-1, 1:-1] += jx * dxl[None, :]
    y[1:-1, 1:-1] += jy * dyl[:, None]
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def naca_thickness(xc: np.ndarray, t: float = 0.10) -> np.ndarray:
    """Half thickness of a symmetric NACA 4-digit section, closed trailing
    edge variant (last coefficient -0.1036 so that y(1) = 0)."""
    return 5.0 * t * (0.2969 * np.sqrt(xc) - 0.1260 * xc - 0.3516 * xc ** 2
                      + 0.2843 * xc ** 3 - 0.1036 * xc ** 4)


def cgrid(ni: int = 256, nj: int = 128, n_wake: int = 32, t: float = 0.10,
          r_outer: float = 20.0, wall_spacing: float = 1e-6,
          bl_fraction: float = 0.5, bl_height: float = 0.05,
          max_aspect: float = 1e4):
    """Algebraic C-grid around a symmetric NACA 4-digit section.

    * airfoil: ``ni - 2*n_wake`` cells, cosine clustered per surface;
    * wake: ``n_wake`` cells per leg from the trailing edge to
      x = 1 + r_outer, geometric from the trailing-edge spacing;
    * outer boundary: half circle of radius ``r_outer`` about (1, 0)
      joined to the straight wake outflow boundaries at y = -+r_outer;
    * j-lines are straight from wall to outer boundary; the inner
      ``bl_fraction`` of the cells is geometric from ``wall_spacing``
      up to ``bl_height`` chords, the rest stretches to the outer boundary;
      along the wake the first normal spacing grows with the streamwise
      spacing so that the cell aspect ratio stays below ``max_aspect``.
    """
    n_af = ni - 2 * n_wake
    if n_af <= 0 or n_af % 2:
        raise ValueError("ni - 2*n_wake must be positive and even")
    ns = n_af // 2
    k = np.arange(ns + 1)
    xl = 0.5 * (1.0 + np.cos(np.pi * k / ns))           # TE -> LE
    xl[0], xl[-1] = 1.0, 0.0
    yl = -naca_thickness(xl, t)
    yl[0] = 0.0
    yl[-1] = 0.0
    # the upper surface is the exact mirror image of the lower one
    x_af = np.concatenate([xl, xl[::-1][1:]])
    y_af = np.concatenate([yl, -yl[::-1][1:]])
    # wake, trailing edge -> outflow
    d_te = x_af[0] - x_af[1]
    dw = _geometric_spacing(n_wake, d_te, r_outer)
    xw = 1.0 + np.concatenate([[0.0], np.cumsum(dw)])
    xw[-1] = 1.0 + r_outer
    x_in = np.concatenate([xw[::-1], x_af[1:-1], xw])
    y_in = np.concatenate([np.zeros(n_wake + 1), y_af[1:-1], np.zeros(n_wake + 1)])
    assert x_in.size == ni + 1
    # outer boundary
    th = -0.5 * np.pi - np.pi * np.arange(ns + 1) / n_af     # lower half
    xo_l = 1.0 + r_outer * np.cos(th)
    yo_l = r_outer * np.sin(th)
    yo_l[-1] = 0.0
    xo_af = np.concatenate([xo_l, xo_l[::-1][1:]])
    yo_af = np.concatenate([yo_l, -yo_l[::-1][1:]])
    x_out = np.concatenate([xw[::-1], xo_af[1:-1], xw])
    y_out = np.concatenate([np.full(n_wake + 1, -r_outer), yo_af[1:-1],
                            np.full(n_wake + 1, r_outer)])
    # normal distribution (fraction of the line length)
    nbl = int(round(nj * bl_fraction))
    length = np.hypot(x_out - x_in, y_out - y_in)
    ds_stream = np.zeros(ni + 1)
    ds_stream[:n_wake + 1] = np.abs(np.gradient(x_in[:n_wake + 1]))
    ds_stream[ni - n_wake:] = np.abs(np.gradient(x_in[ni - n_wake:]))
    first = np.maximum(wall_spacing, ds_stream / max_aspect)
    # far down a short wake the aspect-ratio floor can exceed what a
    # stretched boundary-layer block of nbl cells holds; halve the block's
    # mean spacing there (other columns are left as they are)
    too_big = first * nbl >= bl_height
    first = np.where(too_big, 0.5 * bl_height / max(nbl, 1), first)
    x = np.empty((nj + 1, ni + 1))
    y = np.empty((nj + 1, ni + 1))
    for I in range(ni + 1):
        L = length[I]
        d1 = _geometric_spacing(nbl, first[I] / L, bl_height / L)
        d2 = _geometric_spacing(nj - nbl, d1[-1], 1.0 - bl_height / L)
        eta = np.concatenate([[0.0], np.cumsum(np.concatenate([d1, d2]))])
        eta[-1] = 1.0
        x[:, I] = x_in[I] + (x_out[I] - x_in[I]) * eta
        y[:, I] = y_in[I] + (y_out[I] - y_in[I]) * eta
    # exact mirror symmetry about y = 0: node (ni - I, J) mirrors (I, J);
    # this also makes the wake-cut nodes coincide pairwise
    half = ni // 2
    x[:, ni - half:] = x[:, :half + 1][:, ::-1]
    y[:, ni - half:] = -y[:, :half + 1][:, ::-1]
    y[:, half] = np.where(np.abs(y[:, half]) < 1e-300, 0.0, y[:, half])
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def max_aspect_ratio(x: np.ndarray, y: np.ndarray) -> float:
    """Largest ratio of the cell's mean i-edge to mean j-edge length (or
    inverse), a descriptive statistic of a generated grid."""
    di = 0.5 * (np.hypot(np.diff(x[:-1], axis=1), np.diff(y[:-1], axis=1))
                + np.hypot(np.diff(x[1:], axis=1), np.diff(y[1:], axis=1)))
    dj = 0.5 * (np.hypot(np.diff(x[:, :-1], axis=0), np.diff(y[:, :-1], axis=0))
                + np.hypot(np.diff(x[:, 1:], axis=0), np.diff(y[:, 1:], axis=0)))
    ar = np.maximum(di / dj, dj / di)
    return float(ar.max())


# --------------------------------------------------------------------------
# initial states
# --------------------------------------------------------------------------
def primitive_to_conservative(rho, vx, vy, p, gamma: float = GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
    return np.ascontiguousarray(np.stack([rho, rho * vx, rho * vy, E]))


def uniform_state(ni: int, nj: int, mach: float, alpha_deg: float,
                  gamma: float = GAMMA):
    """Uniform free stream rho=1, p=1, |v| = M*sqrt(gamma) at angle alpha."""
    V = mach * math.sqrt(gamma)
    a = math.radians(alpha_deg)
    one = np.ones((nj, ni))
    return primitive_to_conservative(one, V * math.cos(a) * one,
                                     V * math.sin(a) * one, one, gamma)


def cell_centroids(x: np.ndarray, y: np.ndarray):
    xc = 0.25 * (x[:-1, :-1] + x[:-1, 1:] + x[1:, :-1] + x[1:, 1:])
    yc = 0.25 * (y[:-1, :-1] + y[:-1, 1:] + y[1:, :-1] + y[1:, 1:])
    return xc, yc


def box_initial_state(x: np.ndarray, y: np.ndarray, mach: float = 0.8,
                      alpha_deg: float = 0.0, bump: float = 0.05,
                      width: float = 0.1, noise: float = 1e-3, seed: int = 2,
                      gamma: float = GAMMA):
    """Free stream with a Gaussian density bump and velocity noise, p = 1."""
    xc, yc = cell_centroids(x, y)
    rho = 1.0 + bump * np.exp(-((xc - 0.5) ** 2 + (yc - 0.5) ** 2) / (2 * width ** 2))
    V = mach * math.sqrt(gamma)
    a = math.radians(alpha_deg)
    rng = np.random.default_rng(seed)
    vx = V * math.cos(a) + rng.uniform(-noise, noise, size=xc.shape)
    vy = V * math.sin(a) + rng.uniform(-noise, noise, size=xc.shape)
    return primitive_to_conservative(rho, vx, vy, np.ones_like(rho), gamma)


def perturbed_state(u: np.ndarray, amp: float, seed: int):
    """u * (1 + U(-amp, amp)) component-wise (test inputs)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(u * (1.0 + rng.uniform(-amp, amp, size=u.shape)))


# --------------------------------------------------------------------------
# workload descriptions
# --------------------------------------------------------------------------
@dataclass
class Case:
    name: str
    topology: int
    ni: int
    nj: int
    n_wake: int
    mach: float
    alpha_deg: float
    reynolds: float
    rans: bool
    n_levels: int
    seed: int
    extra: dict = field(default_factory=dict)

    def grid(self):
        if self.topology == BOX:
            return box_grid(self.ni, self.nj, seed=self.seed)
        return cgrid(self.ni, self.nj, self.n_wake)

    def initial_state(self, x, y):
        if self.topology == BOX:
            return box_initial_state(x, y, self.mach, self.alpha_deg,
                                     seed=self.extra.get("state_seed", 2))
        return uniform_state(self.ni, self.nj, self.mach, self.alpha_deg)


def box_case(ni: int = 64, nj: int = 64) -> Case:
    """Euler box: 64x64, wall-side stretching 1.1, 5 % jitter (seed 1),
    M = 0.8 bump + noise (seed 2), single grid."""
    return Case("box_euler_%dx%d" % (ni, nj), BOX, ni, nj, 0, 0.8, 0.0, 0.0,
                False, 1, 1, {"state_seed": 2})


def steady_cgrid_case(ni: int = 256, nj: int = 128, n_wake: int = 32,
                      seed: int = 3, n_levels: int = 3) -> Case:
    """Steady RANS C-grid: Re = 1e7, M = 0.8, alpha ~ U[0, 2] deg (seeded)."""
    rng = np.random.default_rng(seed)
    alpha = float(rng.uniform(0.0, 2.0))
    return Case("cgrid_rans_%dx%d" % (ni, nj), CGRID, ni, nj, n_wake, 0.8,
                alpha, 1e7, True, n_levels, seed)


def batch_cases(n: int = 64, seed: int = 4, n_levels: int = 3):
    """Uneven batch: ni = 16*U{8..32}, nj = 16*U{4..16}, M ~ U[0.5, 0.85],
    alpha ~ U[0, 3] deg, Re = 1e7, RANS."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n):
        ni = 16 * int(rng.integers(8, 33))
        nj = 16 * int(rng.integers(4, 17))
        mach = float(rng.uniform(0.5, 0.85))
        alpha = float(rng.uniform(0.0, 3.0))
        nw = ni // 8
        nw -= nw % 4
        out.append(Case("batch%02d_%dx%d" % (c, ni, nj), CGRID, ni, nj, nw, mach,
                        alpha, 1e7, True, n_levels, seed))
    return out
