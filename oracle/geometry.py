"""Grid metrics of the cell-centred finite-volume discretisation.

Follows the paper's Section 2 (cell-centred finite volumes on a structured
(i, j) mesh) and Section 3 (coarse levels by agglomerating 2x2 cells).

Face vectors
    i-face (I, j), between cells (I-1, j) and (I, j):  S = ( dy, -dx ) of the
    edge node(I, j) -> node(I, j+1); it points towards +i.
    j-face (i, J), between cells (i, J-1) and (i, J):  S = (-dy,  dx ) of the
    edge node(i, J) -> node(i+1, J); it points towards +j.
Cell volume  Omega = 1/2 (d1 x d2) with the diagonals d1 = SW->NE and
    d2 = SE->NW; positive for the right-handed grids used here.
Coarse level: every second node; a coarse face vector equals the sum of its
    two child face vectors, the coarse volume is the sum of the four child
    volumes (agglomeration).

Ghost cells (two layers, needed by the JST stencil) get geometry from the
interior cell they mirror: the same mean face vectors, and a centre
reflected across the boundary face; across the C-grid wake cut the ghost is
the partner cell itself.
"""
from __future__ import annotations

import numpy as np

NG = 2          # ghost layers
BOX, CGRID = 0, 1


def _reflect(cx, cy, mx, my, sx, sy):
    ln = np.sqrt(sx * sx + sy * sy)
    nx = sx / ln
    ny = sy / ln
    dist = (cx - mx) * nx + (cy - my) * ny
    return cx - 2.0 * dist * nx, cy - 2.0 * dist * ny


class Level:
    """Geometry of one multigrid level (interior ni x nj cells)."""

    def __init__(self, x, y, topology: int, n_wake: int, vol=None):
        # node coordinates may be complex (complex-step derivatives with
        # respect to the grid); every metric is then complex as well
        dt = np.result_type(np.asarray(x), np.asarray(y), np.float64)
        self.x = np.asarray(x, dtype=dt)
        self.y = np.asarray(y, dtype=dt)
        self.nj = self.x.shape[0] - 1
        self.ni = self.x.shape[1] - 1
        self.topology = topology
        self.n_wake = n_wake if topology == CGRID else 0
        x, y = self.x, self.y
        ni, nj = self.ni, self.nj
        dxj = x[1:, :] - x[:-1, :]
        dyj = y[1:, :] - y[:-1, :]
        self.Sxi = np.stack([dyj, -dxj])              # (2, nj, ni+1)
        dxi = x[:, 1:] - x[:, :-1]
        dyi = y[:, 1:] - y[:, :-1]
        self.Seta = np.stack([-dyi, dxi])             # (2, nj+1, ni)
        if vol is None:
            d1x = x[1:, 1:] - x[:-1, :-1]
            d1y = y[1:, 1:] - y[:-1, :-1]
            d2x = x[1:, :-1] - x[:-1, 1:]
            d2y = y[1:, :-1] - y[:-1, 1:]
            vol = 0.5 * (d1x * d2y - d1y * d2x)
        if np.any(np.real(vol) <= 0.0):
            raise ValueError("non-positive cell volume (grid must be right-handed)")
        self.vol = vol
        # face midpoints
        self.mxi = (0.5 * (x[:-1, :] + x[1:, :]), 0.5 * (y[:-1, :] + y[1:, :]))
        self.meta = (0.5 * (x[:, :-1] + x[:, 1:]), 0.5 * (y[:, :-1] + y[:, 1:]))
        # padded cell data: centre and mean face vectors
        P = NG
        shape = (nj + 2 * P, ni + 2 * P)
        xc = np.zeros(shape, dtype=dt)
        yc = np.zeros(shape, dtype=dt)
        sb = np.zeros((4,) + shape, dtype=dt)     # sbar_xi x,y ; sbar_eta x,y
        vp = np.zeros(shape, dtype=dt)            # volume, ghosts copy their source
        xc[P:P + nj, P:P + ni] = 0.25 * (((x[:-1, :-1] + x[:-1, 1:]) + x[1:, 1:]) + x[1:, :-1])
        yc[P:P + nj, P:P + ni] = 0.25 * (((y[:-1, :-1] + y[:-1, 1:]) + y[1:, 1:]) + y[1:, :-1])
        sb[0, P:P + nj, P:P + ni] = 0.5 * (self.Sxi[0][:, :-1] + self.Sxi[0][:, 1:])
        sb[1, P:P + nj, P:P + ni] = 0.5 * (self.Sxi[1][:, :-1] + self.Sxi[1][:, 1:])
        sb[2, P:P + nj, P:P + ni] = 0.5 * (self.Seta[0][:-1, :] + self.Seta[0][1:, :])
        sb[3, P:P + nj, P:P + ni] = 0.5 * (self.Seta[1][:-1, :] + self.Seta[1][1:, :])
        vp[P:P + nj, P:P + ni] = vol
        # ghost rows (j), columns i in [0, ni)
        for i in range(ni):
            cut = self.is_cut_column(i)
            for k in range(P):
                jg = P - 1 - k               # padded row of j = -1-k
                if cut:
                    src = (P + k, P + ni - 1 - i)
                    xc[jg, P + i] = xc[src]
                    yc[jg, P + i] = yc[src]
                else:
                    src = (P + k, P + i)
                    xc[jg, P + i], yc[jg, P + i] = _reflect(
                        xc[src], yc[src], self.meta[0][0, i], self.meta[1][0, i],
                        self.Seta[0][0, i], self.Seta[1][0, i])
                sb[:, jg, P + i] = sb[:, src[0], src[1]]
                vp[jg, P + i] = vp[src]
                jt = P + nj + k              # padded row of j = nj+k
                src = (P + nj - 1 - k, P + i)
                xc[jt, P + i], yc[jt, P + i] = _reflect(
                    xc[src], yc[src], self.meta[0][nj, i], self.meta[1][nj, i],
                    self.Seta[0][nj, i], self.Seta[1][nj, i])
                sb[:, jt, P + i] = sb[:, src[0], src[1]]
                vp[jt, P + i] = vp[src]
        # ghost columns (i), every padded row (corners from the ghost rows)
        for jp in range(nj + 2 * P):
            jc = min(max(jp - P, 0), nj - 1)
            for k in range(P):
                ig = P - 1 - k
                src = (jp, P + k)
                xc[jp, ig], yc[jp, ig] = _reflect(
                    xc[src], yc[src], self.mxi[0][jc, 0], self.mxi[1][jc, 0],
                    self.Sxi[0][jc, 0], self.Sxi[1][jc, 0])
                sb[:, jp, ig] = sb[:, src[0], src[1]]
                vp[jp, ig] = vp[src]
                ie = P + ni + k
                src = (jp, P + ni - 1 - k)
                xc[jp, ie], yc[jp, ie] = _reflect(
                    xc[src], yc[src], self.mxi[0][jc, ni], self.mxi[1][jc, ni],
                    self.Sxi[0][jc, ni], self.Sxi[1][jc, ni])
                sb[:, jp, ie] = sb[:, src[0], src[1]]
                vp[jp, ie] = vp[src]
        self.xc, self.yc, self.sbar, self.volp = xc, yc, sb, vp
        # grid velocities of a moving (rigidly rotating) mesh; None: fixed
        self.wxi = self.weta = self.wc = None
        # wall (or cut) distance: cell centre to the midpoint of face (i, J=0)
        self.wall_dist = np.sqrt(
            (xc[P:P + nj, P:P + ni] - self.meta[0][0][None, :]) ** 2
            + (yc[P:P + nj, P:P + ni] - self.meta[1][0][None, :]) ** 2)

    # ------------------------------------------------------------------
    def is_cut_column(self, i: int) -> bool:
        return self.topology == CGRID and (i < self.n_wake or i >= self.ni - self.n_wake)

    def cut_mask(self) -> np.ndarray:
        i = np.arange(self.ni)
        if self.topology != CGRID:
            return np.zeros(self.ni, dtype=bool)
        return (i < self.n_wake) | (i >= self.ni - self.n_wake)

    def coarsen(self) -> "Level":
        if self.ni % 2 or self.nj % 2 or (self.topology == CGRID and self.n_wake % 2):
            raise ValueError("level cannot be agglomerated 2x2")
        v = self.vol
        vc = ((v[0::2, 0::2] + v[0::2, 1::2]) + v[1::2, 0::2]) + v[1::2, 1::2]
        return Level(self.x[::2, ::2], self.y[::2, ::2], self.topology,
                     self.n_wake // 2, vol=vc)


def rotated(lev: Level, theta: float, omega: float, px: float, py: float) -> Level:
    """The level rigidly rotated by theta (radians, counter-clockwise)
    about (px, py) and spinning at omega (radians per unit time): face
    vectors, mean face vectors, centres and face midpoints rotate, volumes
    and wall distances do not.  Grid velocities omega x (r - pivot) are
    attached at the face midpoints (wxi, weta) and at the padded cell
    centres (wc) for the moving-mesh (ALE) terms."""
    import copy
    import math
    c, s = math.cos(theta), math.sin(theta)

    def vec(vx, vy):
        return c * vx - s * vy, s * vx + c * vy

    def pt(x, y):
        dx, dy = x - px, y - py
        return px + (c * dx - s * dy), py + (s * dx + c * dy)

    r = copy.copy(lev)
    r.x, r.y = pt(lev.x, lev.y)
    r.Sxi = np.stack(vec(lev.Sxi[0], lev.Sxi[1]))
    r.Seta = np.stack(vec(lev.Seta[0], lev.Seta[1]))
    sb0, sb1 = vec(lev.sbar[0], lev.sbar[1])
    sb2, sb3 = vec(lev.sbar[2], lev.sbar[3])
    r.sbar = np.stack([sb0, sb1, sb2, sb3])
    r.xc, r.yc = pt(lev.xc, lev.yc)
    r.mxi = pt(lev.mxi[0], lev.mxi[1])
    r.meta = pt(lev.meta[0], lev.meta[1])

    def gv(x, y):
        return -omega * (y - py), omega * (x - px)

    r.wxi = gv(*r.mxi)
    r.weta = gv(*r.meta)
    r.wc = gv(r.xc, r.yc)
    return r


def build_levels(x, y, topology: int, n_wake: int, n_levels: int):
    """Levels ordered fine -> coarse (index 0 is the finest)."""
    lev = [Level(x, y, topology, n_wake)]
    for _ in range(n_levels - 1):
        lev.append(lev[-1].coarsen())
    return lev
