"""Spatial residual: JST convective flux with scalar artificial dissipation,
viscous fluxes from vertex-centred dual grids, the Baldwin-Lomax eddy
viscosity, and the split F = f^c + f^v used by the additive smoothers.

Paper passages followed:
* Section 2, JST flux: the face flux averages the two cell fluxes and the
  dissipation d = eps2 dw - eps4 (dw_{j+1} - 2 dw_j + dw_{j-1}) acts on
  w = (rho, rho v, rho H); eps2 = s r (eq. "e2"), eps4 = max(0, r/32 - 2 eps2)
  (eq. "e4"), s_{j+1/2} = min(0.25, max(s_j, s_{j+1})); entropy sensor
  S = p / rho^gamma for RANS, pressure sensor for Euler; r = |v_n| + a with
  the face value max(r_j, r_{j+1}) and the multidimensional correction of
  eq. "spectralcorrection".
  Readings: the dissipation is subtracted from the central flux (the sign
  that makes it dissipative); the sensor denominator is
  S_{j+1} + 2 S_j + S_{j-1} + 0.001; r uses the cell's mean face vector so
  that it carries the face length; through a solid wall face the
  convective flux is the pressure force p_w S alone (no mass, momentum or
  energy transport through the wall) with p_w the mean of the wall cell and
  its ghost, and there is no artificial dissipation.
* Section 2, viscous terms: velocity and temperature gradients on dual
  cells around vertices (Green-Gauss over the quadrilateral of the four
  surrounding cell centres); a face gradient is the mean of its two end
  vertices. Heat flux (mu/Pr + mu_t/Pr_t) grad h, h = gamma/(gamma-1) p/rho.
  Reading: Sutherland's law for mu, Pr_t = 0.9.
* Section 2, Baldwin-Lomax algebraic eddy viscosity, standard constants of
  the cited model (A+ = 26, C_cp = 1.6, C_kleb = 0.3, C_wk = 0.25,
  kappa = 0.4, K = 0.0168), evaluated on the fine level.
* Section 3: coarse levels use a first-order JST flux (no fourth
  difference, no sensor): eps2 = kappa2c * r (reading, kappa2c = 0.125);
  they keep the viscous flux with the restricted eddy viscosity (reading).
* Section 4.1, eq. "split-rhs": f^c holds the convective fluxes, the
  physical time derivative and the multigrid source; f^v the artificial
  dissipation and the viscous terms.
* Eq. "nonlin-eq" / "nonlin-eq-steady": F = Omega^-1 f (+ BDF2 term).
"""
from __future__ import annotations

import numpy as np

from . import gas
from .bc import fill_scalar_ghosts
from .geometry import NG, BOX, CGRID

GAMMA = gas.GAMMA
SUTH = 110.4 / 288.15
BL_APLUS, BL_CCP, BL_CKLEB, BL_CWK, BL_KAPPA, BL_K = 26.0, 1.6, 0.3, 0.25, 0.4, 0.0168


def _abs(x):
    """|x|; for complex arguments (complex-step differentiation) the value
    times the sign of its real part, which carries the derivative."""
    if np.iscomplexobj(x):
        return np.where(x.real < 0.0, -x, x)
    return np.abs(x)


def _max(a, b):
    """max(a, b); for complex arguments (complex-step differentiation) the
    branch whose real part is larger, the first argument on ties (the
    derivative of the taken branch)."""
    if np.iscomplexobj(a) or np.iscomplexobj(b):
        return np.where(np.real(b) > np.real(a), b, a)
    return np.maximum(a, b)


def _min(a, b):
    """min(a, b) with the tie rule of _max."""
    if np.iscomplexobj(a) or np.iscomplexobj(b):
        return np.where(np.real(b) < np.real(a), b, a)
    return np.minimum(a, b)


def _cbrt(x):
    """Real cube root; for complex arguments its first-order extension
    cbrt(a) + i b / (3 cbrt(a)^2) (complex-step differentiation)."""
    if np.iscomplexobj(x):
        c = np.cbrt(x.real)
        return c + 1j * (x.imag / (3.0 * c * c))
    return np.cbrt(x)


def sutherland(T, mu_inf):
    return ((mu_inf * (T * np.sqrt(T))) * (1.0 + SUTH)) / (T + SUTH)


def cell_scalars(lev, Up, rans: bool):
    """Pressure, sensor quantity and corrected spectral radii on the padded
    array (all cells, ghosts included)."""
    rho = Up[0]
    vx = Up[1] / rho
    vy = Up[2] / rho
    p = gas.pressure(Up)
    a = np.sqrt(GAMMA * p / rho)
    q = p / rho ** GAMMA if rans else p
    sb = lev.sbar
    vnx = vx * sb[0] + vy * sb[1]
    vne = vx * sb[2] + vy * sb[3]
    if lev.wc is not None:         # moving mesh: velocity relative to the cell
        vnx = vnx - (lev.wc[0] * sb[0] + lev.wc[1] * sb[1])
        vne = vne - (lev.wc[0] * sb[2] + lev.wc[1] * sb[3])
    rxi = _abs(vnx) + a * np.sqrt(sb[0] * sb[0] + sb[1] * sb[1])
    reta = _abs(vne) + a * np.sqrt(sb[2] * sb[2] + sb[3] * sb[3])
    t = reta / rxi
    rtxi = rxi * (1.0 + _cbrt(t * t))
    t = rxi / reta
    rteta = reta * (1.0 + _cbrt(t * t))
    return p, q, rxi, reta, rtxi, rteta


def local_time_step(lev, Up, cfl: float, dt_form: int = 1):
    """Pseudo time step per cell, a reading of "c* times the local mesh
    width" (Section 4.1): the directional CFL steps Omega / r_xi and
    Omega / r_eta (r carries the face length, so Omega / r is a width over
    a wave speed); dt_form 1 takes the smaller of the two, c* Omega /
    max(r_xi, r_eta), which on a Cartesian cell at zero incidence is the
    step c* dx / (|v_1| + a) of the Fourier analysis; dt_form 0 takes
    c* Omega / (r_xi + r_eta)."""
    p, q, rxi, reta, _, _ = cell_scalars(lev, Up, False)
    P = NG
    rx = rxi[P:-P, P:-P]
    re = reta[P:-P, P:-P]
    r = np.maximum(rx, re) if dt_form else rx + re
    return cfl * lev.vol / r


def _sensor(q_m, q_0, q_p):
    num = (q_p - 2.0 * q_0) + q_m
    den = ((q_p + 2.0 * q_0) + q_m) + 0.001
    return _abs(num / den)


def _face_dissipation(wLL, wL, wR, wRR, sL, sR, rL, rR, second_order: bool, kappa2c: float):
    rf = _max(rL, rR)
    if second_order:
        sf = _min(0.25, _max(sL, sR))
        e2 = sf * rf
        e4 = _max(0.0, rf / 32.0 - 2.0 * e2)
        return e2 * (wR - wL) - e4 * (((wRR - 3.0 * wR) + 3.0 * wL) - wLL)
    e2 = kappa2c * rf
    return e2 * (wR - wL)


def convective_faces(lev, Up, par, second_order: bool):
    """Central flux C and dissipation d on every i-face (I = 0..ni) and
    j-face (J = 0..nj); arrays (4, nj, ni+1) and (4, nj+1, ni)."""
    P = NG
    ni, nj = lev.ni, lev.nj
    rans = par.model == 1
    p, q, rxi, reta, rtxi, rteta = cell_scalars(lev, Up, rans)
    w = Up.copy()
    w[3] = Up[3] + p
    # i-faces: rows interior, L = I-1, R = I
    rows = slice(P, P + nj)
    sl = lambda o: slice(P - 2 + o, P - 2 + o + ni + 1)   # o=0: LL, 1: L, 2: R, 3: RR
    sx, sy = lev.Sxi[0], lev.Sxi[1]
    UL, UR = Up[:, rows, sl(1)], Up[:, rows, sl(2)]
    pL, pR = p[rows, sl(1)], p[rows, sl(2)]
    Cxi = 0.5 * (gas.normal_flux(UL, pL, sx, sy) + gas.normal_flux(UR, pR, sx, sy))
    if lev.wxi is not None:        # moving face: - (w . S) times the mean state
        qxi = lev.wxi[0] * sx + lev.wxi[1] * sy
        Cxi = Cxi - qxi * (0.5 * (UL + UR))
    sxi = None
    if second_order:
        s = np.zeros_like(q)
        s[:, 1:-1] = _sensor(q[:, :-2], q[:, 1:-1], q[:, 2:])
        sxi = s
    Dxi = _face_dissipation(w[:, rows, sl(0)], w[:, rows, sl(1)], w[:, rows, sl(2)],
                            w[:, rows, sl(3)],
                            sxi[rows, sl(1)] if second_order else None,
                            sxi[rows, sl(2)] if second_order else None,
                            rtxi[rows, sl(1)], rtxi[rows, sl(2)], second_order, par.kappa2c)
    # j-faces: columns interior, L = J-1, R = J
    cols = slice(P, P + ni)
    sj = lambda o: slice(P - 2 + o, P - 2 + o + nj + 1)
    sx, sy = lev.Seta[0], lev.Seta[1]
    UL, UR = Up[:, sj(1), cols], Up[:, sj(2), cols]
    pL, pR = p[sj(1), cols], p[sj(2), cols]
    Ceta = 0.5 * (gas.normal_flux(UL, pL, sx, sy) + gas.normal_flux(UR, pR, sx, sy))
    qeta = None
    if lev.weta is not None:
        qeta = lev.weta[0] * sx + lev.weta[1] * sy
        Ceta = Ceta - qeta * (0.5 * (UL + UR))
    seta = None
    if second_order:
        s = np.zeros_like(q)
        s[1:-1, :] = _sensor(q[:-2, :], q[1:-1, :], q[2:, :])
        seta = s
    Deta = _face_dissipation(w[:, sj(0), cols], w[:, sj(1), cols], w[:, sj(2), cols],
                             w[:, sj(3), cols],
                             seta[sj(1), cols] if second_order else None,
                             seta[sj(2), cols] if second_order else None,
                             rteta[sj(1), cols], rteta[sj(2), cols], second_order, par.kappa2c)
    # solid-wall faces: no flow through the wall, so the convective flux
    # is the pressure force alone (mean of the cell and its mirror ghost),
    # and no artificial dissipation
    wallcols = ~lev.cut_mask()
    pw = 0.5 * (p[P - 1, cols] + p[P, cols])
    Ceta[0, 0, wallcols] = 0.0
    Ceta[1, 0, wallcols] = (pw * sx[0])[wallcols]
    Ceta[2, 0, wallcols] = (pw * sy[0])[wallcols]
    # a moving wall does the pressure work p_w (w . S)
    Ceta[3, 0, wallcols] = 0.0 if qeta is None else (pw * qeta[0])[wallcols]
    Deta[:, 0, wallcols] = 0.0
    return Cxi, Dxi, Ceta, Deta


def vertex_gradients(lev, phis):
    """Green-Gauss gradients at every vertex (J = 0..nj, I = 0..ni) over the
    quadrilateral SW -> SE -> NE -> NW of the surrounding cell centres.
    ``phis``: list of padded cell fields; returns list of (gx, gy)."""
    P = NG
    ni, nj = lev.ni, lev.nj
    J0 = slice(P - 1, P + nj)        # rows j-1 for J = 0..nj
    J1 = slice(P, P + nj + 1)
    I0 = slice(P - 1, P + ni)
    I1 = slice(P, P + ni + 1)
    corners = [(J0, I0), (J0, I1), (J1, I1), (J1, I0)]     # SW, SE, NE, NW
    X = [lev.xc[c] for c in corners]
    Y = [lev.yc[c] for c in corners]
    A = 0.5 * ((X[2] - X[0]) * (Y[3] - Y[1]) - (Y[2] - Y[0]) * (X[3] - X[1]))
    out = []
    for phi in phis:
        F = [phi[c] for c in corners]
        gx = None
        gy = None
        for e in range(4):
            a, b = e, (e + 1) % 4
            m = 0.5 * (F[a] + F[b])
            tx = m * (Y[b] - Y[a])
            ty = m * (X[a] - X[b])
            gx = tx if gx is None else gx + tx
            gy = ty if gy is None else gy + ty
        out.append((gx / A, gy / A))
    return out


def viscous_faces(lev, Up, mutp, par):
    """Viscous flux dotted with the face vector on every i- and j-face."""
    P = NG
    ni, nj = lev.ni, lev.nj
    rho = Up[0]
    vx = Up[1] / rho
    vy = Up[2] / rho
    T = gas.pressure(Up) / rho
    (ux, uy), (wx, wy), (Tx, Ty) = vertex_gradients(lev, [vx, vy, T])
    mu_inf = par.mach * np.sqrt(GAMMA) / par.reynolds
    cp = GAMMA / (GAMMA - 1.0)

    def face(gL, gR, cL, cR, sx, sy):
        # gL/gR: vertex slices of the two end vertices, cL/cR: cell slices
        fux = 0.5 * (ux[gL] + ux[gR])
        fuy = 0.5 * (uy[gL] + uy[gR])
        fwx = 0.5 * (wx[gL] + wx[gR])
        fwy = 0.5 * (wy[gL] + wy[gR])
        fTx = 0.5 * (Tx[gL] + Tx[gR])
        fTy = 0.5 * (Ty[gL] + Ty[gR])
        fvx = 0.5 * (vx[cL] + vx[cR])
        fvy = 0.5 * (vy[cL] + vy[cR])
        fT = 0.5 * (T[cL] + T[cR])
        mu = sutherland(fT, mu_inf)
        mut = 0.5 * (mutp[cL] + mutp[cR])
        mue = mu + mut
        k = (mu / par.prandtl + mut / par.prandtl_t) * cp
        div = fux + fwy
        txx = mue * (2.0 * fux - (2.0 / 3.0) * div)
        tyy = mue * (2.0 * fwy - (2.0 / 3.0) * div)
        txy = mue * (fuy + fwx)
        qx = k * fTx
        qy = k * fTy
        g0 = np.zeros_like(txx)
        g1 = txx * sx + txy * sy
        g2 = txy * sx + tyy * sy
        g3 = ((fvx * txx + fvy * txy) + qx) * sx + ((fvx * txy + fvy * tyy) + qy) * sy
        return np.stack([g0, g1, g2, g3])

    rows = slice(P, P + nj)
    # i-face (I, j): vertices (I, j), (I, j+1); cells (I-1, j), (I, j)
    Gxi = face((slice(0, nj), slice(0, ni + 1)), (slice(1, nj + 1), slice(0, ni + 1)),
               (rows, slice(P - 1, P + ni)), (rows, slice(P, P + ni + 1)),
               lev.Sxi[0], lev.Sxi[1])
    cols = slice(P, P + ni)
    # j-face (i, J): vertices (i, J), (i+1, J); cells (i, J-1), (i, J)
    Geta = face((slice(0, nj + 1), slice(0, ni)), (slice(0, nj + 1), slice(1, ni + 1)),
                (slice(P - 1, P + nj), cols), (slice(P, P + nj + 1), cols),
                lev.Seta[0], lev.Seta[1])
    return Gxi, Geta


def baldwin_lomax(lev, Up, par):
    """Eddy viscosity per interior cell, column by column along the j-lines
    from the wall (or from the wake cut, where the wall damping is dropped).

    Readings: vorticity at a cell centre = mean of its four vertex values;
    the wall quantities are those of the first cell; the search for F_max,
    U_dif and the inner/outer crossover is limited to the inner half of the
    j-cells (the boundary-layer half of the grid); first maximum and first
    crossover win ties."""
    P = NG
    ni, nj = lev.ni, lev.nj
    rho = Up[0]
    vx = Up[1] / rho
    vy = Up[2] / rho
    T = gas.pressure(Up) / rho
    (ux, uy), (wx, wy) = vertex_gradients(lev, [vx, vy])
    om_v = wx - uy
    om = np.abs(0.25 * (((om_v[:-1, :-1] + om_v[:-1, 1:]) + om_v[1:, 1:]) + om_v[1:, :-1]))
    mu_inf = par.mach * np.sqrt(GAMMA) / par.reynolds
    r = rho[P:P + nj, P:P + ni]
    speed = np.sqrt(vx[P:P + nj, P:P + ni] ** 2 + vy[P:P + nj, P:P + ni] ** 2)
    y = lev.wall_dist
    muw = sutherland(T[P, P:P + ni], mu_inf)
    rhow = r[0]
    tauw = muw * om[0]
    cut = lev.cut_mask()
    yplus = y * np.sqrt(rhow * tauw)[None, :] / muw[None, :]
    damp = 1.0 - np.exp(-yplus / BL_APLUS)
    damp = np.where(cut[None, :], 1.0, damp)
    jb = nj // 2
    F = y * om * damp
    jmax = np.argmax(F[:jb], axis=0)
    cols = np.arange(ni)
    Fmax = F[jmax, cols]
    ymax = y[jmax, cols]
    udif = speed[:jb].max(axis=0) - speed[:jb].min(axis=0)
    safe = np.where(Fmax > 0.0, Fmax, 1.0)
    fwake = np.where(Fmax > 0.0,
                     np.minimum(ymax * Fmax, BL_CWK * ymax * udif * udif / safe), 0.0)
    t = BL_CKLEB * y / ymax[None, :]
    t2 = t * t
    fkleb = 1.0 / (1.0 + 5.5 * (t2 * t2 * t2))
    l = BL_KAPPA * y * damp
    mui = r * (l * l) * om
    muo = r * BL_K * BL_CCP * fwake[None, :] * fkleb
    cross = mui[:jb] >= muo[:jb]
    jc = np.where(cross.any(axis=0), np.argmax(cross, axis=0), jb)
    jj = np.arange(nj)[:, None]
    return np.where(jj < jc[None, :], mui, muo)


def padded_eddy_viscosity(lev, mut):
    P = NG
    mp = np.zeros((lev.nj + 2 * P, lev.ni + 2 * P))
    mp[P:P + lev.nj, P:P + lev.ni] = mut
    return fill_scalar_ghosts(mp, lev)


def split_residual(lev, Up, par, fine: bool, mutp=None, time_src=None, forcing=None):
    """(F^c, F^v), per unit volume, for the padded state Up whose ghosts are
    already filled.  ``time_src`` is the BDF term, ``forcing`` the FAS
    source s of the level (the smoother drives F(u) - s to zero).  RANS
    levels carry the viscous flux with the padded eddy viscosity ``mutp``
    on every level (the fine level's Baldwin-Lomax field, restricted to
    the coarse levels)."""
    ni, nj = lev.ni, lev.nj
    Cxi, Dxi, Ceta, Deta = convective_faces(lev, Up, par, second_order=fine)
    fc = (Cxi[:, :, 1:] - Cxi[:, :, :-1]) + (Ceta[:, 1:, :] - Ceta[:, :-1, :])
    if par.model == 1 and mutp is not None:
        Gxi, Geta = viscous_faces(lev, Up, mutp, par)
        Vxi = -Dxi - Gxi
        Veta = -Deta - Geta
    else:
        Vxi = -Dxi
        Veta = -Deta
    fv = (Vxi[:, :, 1:] - Vxi[:, :, :-1]) + (Veta[:, 1:, :] - Veta[:, :-1, :])
    Fc = fc / lev.vol
    if time_src is not None:
        Fc = Fc + time_src
    if forcing is not None:
        Fc = Fc - forcing
    Fv = fv / lev.vol
    return Fc, Fv
