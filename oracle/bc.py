"""Ghost-cell boundary conditions (Section 2: no-slip walls and far-field
conditions through Riemann invariants).

Two ghost layers; layer k (k = 0, 1 counted from the boundary) takes the
boundary rule applied to interior cell k.

* wall (box bottom, airfoil surface): rho and p mirrored; no-slip
  (RANS) v_g = -v, slip (Euler) v_g = v - 2 (v.n) n with n the unit normal
  of the adjacent boundary face;
* C-grid wake cut: ghost (i, -1-k) is the interior cell (ni-1-i, k);
* far field (box top and sides, C-grid outer boundary and outflow
  planes): one-dimensional Riemann invariants normal to the boundary face;
  entropy and tangential velocity come from the upwind side;
* j-ghost rows are filled first (for interior i); the i-ghost columns are
  then filled for every padded row, which defines the corners.
"""
from __future__ import annotations

import numpy as np

from . import gas
from .geometry import NG, CGRID

GAMMA = gas.GAMMA


def riemann_farfield(Ui, Uinf, nx, ny):
    """Boundary state from the interior state Ui and the free stream for an
    outward unit normal n (subsonic characteristic treatment)."""
    g1 = GAMMA - 1.0
    rho = Ui[0]
    vx = Ui[1] / rho
    vy = Ui[2] / rho
    p = gas.pressure(Ui)
    a = np.sqrt(GAMMA * p / rho)
    rinf = Uinf[0]
    vxf = Uinf[1] / rinf
    vyf = Uinf[2] / rinf
    pf = gas.pressure(Uinf)
    af = np.sqrt(GAMMA * pf / rinf)
    vn = vx * nx + vy * ny
    vnf = vxf * nx + vyf * ny
    rp = vn + 2.0 * a / g1
    rm = vnf - 2.0 * af / g1
    vnb = 0.5 * (rp + rm)
    ab = 0.25 * g1 * (rp - rm)
    out = vnb > 0.0
    s = np.where(out, p / rho ** GAMMA, pf / rinf ** GAMMA)
    tx = np.where(out, vx - vn * nx, vxf - vnf * nx)
    ty = np.where(out, vy - vn * ny, vyf - vnf * ny)
    base = ab * ab / (GAMMA * s)
    rhob = base * base * np.sqrt(base)          # base ** (1/(gamma-1)), gamma = 1.4
    pb = rhob * ab * ab / GAMMA
    ub = tx + vnb * nx
    vb = ty + vnb * ny
    Eb = pb / g1 + 0.5 * rhob * (ub * ub + vb * vb)
    return np.stack([rhob, rhob * ub, rhob * vb, Eb])


def wall_ghost(Ui, nx, ny, noslip: bool):
    rho = Ui[0]
    mx, my = Ui[1], Ui[2]
    if noslip:
        return np.stack([rho, -mx, -my, Ui[3]])
    mn = mx * nx + my * ny
    return np.stack([rho, mx - 2.0 * mn * nx, my - 2.0 * mn * ny, Ui[3]])


def _relative(U, wx, wy):
    """The state seen from a boundary moving at w: velocity v - w, same
    density and pressure."""
    rho = U[0]
    p = gas.pressure(U)
    mx = U[1] - rho * wx
    my = U[2] - rho * wy
    return np.stack([rho, mx, my, p / (GAMMA - 1.0) + 0.5 * (mx * mx + my * my) / rho])


def _absolute(U, wx, wy):
    """Inverse of _relative."""
    rho = U[0]
    p = gas.pressure(U)
    mx = U[1] + rho * wx
    my = U[2] + rho * wy
    return np.stack([rho, mx, my, p / (GAMMA - 1.0) + 0.5 * (mx * mx + my * my) / rho])


def moving_wall_ghost(Ui, nx, ny, wx, wy, noslip: bool):
    """Wall moving at w: no-slip v_g = 2 w - v, slip: the velocity relative
    to the wall mirrored; density and pressure mirrored."""
    rho = Ui[0]
    p = gas.pressure(Ui)
    if noslip:
        mx = 2.0 * rho * wx - Ui[1]
        my = 2.0 * rho * wy - Ui[2]
    else:
        rx = Ui[1] - rho * wx
        ry = Ui[2] - rho * wy
        rn = rx * nx + ry * ny
        mx = (rx - 2.0 * rn * nx) + rho * wx
        my = (ry - 2.0 * rn * ny) + rho * wy
    return np.stack([rho, mx, my, p / (GAMMA - 1.0) + 0.5 * (mx * mx + my * my) / rho])


def _farfield_moving(Ui, uinf, nx, ny, w):
    """Riemann far field for a boundary moving at w (None: fixed)."""
    if w is None:
        return riemann_farfield(Ui, uinf, nx, ny)
    wx, wy = w
    ur = _relative(Ui, wx, wy)
    fr = _relative(np.broadcast_to(uinf, Ui.shape), wx, wy)
    return _absolute(riemann_farfield(ur, fr, nx, ny), wx, wy)


def _unit(sx, sy):
    ln = np.sqrt(sx * sx + sy * sy)
    return sx / ln, sy / ln


def fill_ghosts(Up, lev, Uinf, noslip: bool):
    """Fill both ghost layers of the padded state Up (4, nj+4, ni+4) in place."""
    P = NG
    ni, nj = lev.ni, lev.nj
    uinf = Uinf[:, None]
    cut = lev.cut_mask()
    wall = ~cut
    ii = np.arange(ni)
    # bottom (j < 0)
    nbx, nby = _unit(lev.Seta[0][0], lev.Seta[1][0])          # +j, into the domain
    ntx, nty = _unit(lev.Seta[0][nj], lev.Seta[1][nj])        # +j, out of the domain
    moving = lev.weta is not None
    for k in range(P):
        jg = P - 1 - k
        Ui = Up[:, P + k, P:P + ni]
        if moving:
            g = moving_wall_ghost(Ui, nbx, nby, lev.weta[0][0], lev.weta[1][0], noslip)
        else:
            g = wall_ghost(Ui, nbx, nby, noslip)
        if lev.topology == CGRID:
            partner = Up[:, P + k, P + (ni - 1 - ii)]
            g = np.where(cut[None, :], partner, g)
        Up[:, jg, P:P + ni] = g
        Ui = Up[:, P + nj - 1 - k, P:P + ni]
        wt = (lev.weta[0][nj], lev.weta[1][nj]) if moving else None
        Up[:, P + nj + k, P:P + ni] = _farfield_moving(Ui, uinf, ntx, nty, wt)
    # sides, every padded row
    jc = np.clip(np.arange(nj + 2 * P) - P, 0, nj - 1)
    nwx, nwy = _unit(-lev.Sxi[0][jc, 0], -lev.Sxi[1][jc, 0])  # outward at i = 0
    nex, ney = _unit(lev.Sxi[0][jc, ni], lev.Sxi[1][jc, ni])  # outward at i = ni
    ww = (lev.wxi[0][jc, 0], lev.wxi[1][jc, 0]) if moving else None
    we = (lev.wxi[0][jc, ni], lev.wxi[1][jc, ni]) if moving else None
    for k in range(P):
        Ui = Up[:, :, P + k]
        Up[:, :, P - 1 - k] = _farfield_moving(Ui, uinf, nwx, nwy, ww)
        Ui = Up[:, :, P + ni - 1 - k]
        Up[:, :, P + ni + k] = _farfield_moving(Ui, uinf, nex, ney, we)
    return Up


def fill_scalar_ghosts(sp, lev, wall_value: float = 0.0):
    """Ghost values of a padded cell scalar (the eddy viscosity): zero at
    walls, copied from the mirrored interior cell at far-field boundaries,
    the partner cell across the wake cut."""
    P = NG
    ni, nj = lev.ni, lev.nj
    cut = lev.cut_mask()
    ii = np.arange(ni)
    for k in range(P):
        g = np.full(ni, wall_value)
        if lev.topology == CGRID:
            g = np.where(cut, sp[P + k, P + (ni - 1 - ii)], g)
        sp[P - 1 - k, P:P + ni] = g
        sp[P + nj + k, P:P + ni] = sp[P + nj - 1 - k, P:P + ni]
    for k in range(P):
        sp[:, P - 1 - k] = sp[:, P + k]
        sp[:, P + ni + k] = sp[:, P + ni - 1 - k]
    return sp
