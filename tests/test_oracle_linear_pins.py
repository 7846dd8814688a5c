"""Pins of the oracle's residual pieces against facts that do not come from
the oracle's own formulas (CPU only):

* the linearisation of the fine-level Euler residual about a constant state
  on a uniform Cartesian box, applied to a Fourier mode at interior cells,
  equals the Fourier symbols of the discrete Fourier analysis section
  (H_c for f^c, H_v for f^v; the analysis is pinned separately to the
  printed amplification factors), which pins the central flux, the JST
  fourth-difference stencil and its sign, eps4 = r / 32 with a zero sensor,
  the face-scaled spectral radii with the multidimensional correction of
  eq. "spectralcorrection", and which terms the f^c / f^v split holds;
* the pseudo time step against its closed forms on that box;
* the viscous flux for linear velocity and temperature fields, for which
  the dual-cell gradients are exact, against the Newtonian stress with the
  Stokes hypothesis and Fourier's law, worked out by hand;
* the sensor and the dissipation coefficients at hand-computed values;
* the bilinear prolongation reproducing linear fields;
* the far-field Riemann state keeping the outgoing invariant from the
  interior, the incoming one from the free stream, and entropy and
  tangential velocity from the upwind side.
"""
import dataclasses

import numpy as np
import pytest

import fas_inputs as fi
from oracle import bc, dfa, gas
from oracle import fas as ofas
from oracle import residual as res
from oracle.adjoint import H_CS
from oracle.geometry import NG, build_levels

GAMMA = 1.4


def _uniform_box(ni, nj):
    xs = np.linspace(0.0, 1.0, ni + 1)
    ys = np.linspace(0.0, 1.0, nj + 1)
    x, y = np.meshgrid(xs, ys)
    return x, y


def _linearised_split(ni, nj, U, theta, vhat):
    """(J_c m, J_v m) for the mode m_ij = vhat exp(i (Theta_x i + Theta_y j))
    at the constant state U, by the complex step on its real and imaginary
    parts (two directional derivatives)."""
    x, y = _uniform_box(ni, nj)
    lev = build_levels(x, y, fi.BOX, 0, 1)[0]
    par = ofas.Params(model=0, mach=0.8)
    uinf = gas.freestream(0.8, 0.0)
    jj, ii = np.meshgrid(np.arange(nj), np.arange(ni), indexing="ij")
    phase = np.exp(1j * (theta[0] * ii + theta[1] * jj))
    mode = vhat[:, None, None] * phase[None]
    base = np.broadcast_to(np.asarray(U, dtype=float)[:, None, None], (4, nj, ni))
    outs = []
    for part in (mode.real, mode.imag):
        Up = np.zeros((4, nj + 2 * NG, ni + 2 * NG), dtype=complex)
        Up[:, NG:NG + nj, NG:NG + ni] = base + 1j * H_CS * part
        bc.fill_ghosts(Up, lev, uinf.astype(complex), noslip=False)
        Fc, Fv = res.split_residual(lev, Up, par, True, None, None, None)
        outs.append((Fc.imag / H_CS, Fv.imag / H_CS))
    Jc = outs[0][0] + 1j * outs[1][0]
    Jv = outs[0][1] + 1j * outs[1][1]
    return Jc, Jv, phase


@pytest.mark.parametrize("U,ni,nj,corr", [
    # 45 degrees on square cells: r_xi = r_eta, so the multidimensional
    # correction is exactly 2 in each direction, with no formula involved
    ((1.0, np.sqrt(2.0) / 2.0, np.sqrt(2.0) / 2.0, 3.290), 16, 16, "two"),
    # zero incidence on cells twice as tall as wide: the correction of eq.
    # "spectralcorrection", 1 + (r_other / r)^(2/3), with face-scaled r
    ((1.0, 1.0, 0.0, 3.290), 16, 8, "formula"),
])
def test_linearised_residual_equals_the_fourier_symbols(U, ni, nj, corr):
    U = np.asarray(U)
    v1, v2 = U[1] / U[0], U[2] / U[0]
    a = np.sqrt(GAMMA * gas.pressure(U) / U[0])
    dx, dy = 1.0 / ni, 1.0 / nj
    if corr == "two":
        mx = my = 2.0
    else:
        rx, ry = (abs(v1) + a) * dy, (abs(v2) + a) * dx     # |v . S| + a |S|
        mx = 1.0 + (ry / rx) ** (2.0 / 3.0)
        my = 1.0 + (rx / ry) ** (2.0 / 3.0)
    case = dfa.DfaCase(u=tuple(U), nx=ni, ar=dy / dx, unsteady=False)
    rng = np.random.default_rng(4)
    inner = (slice(3, nj - 3), slice(3, ni - 3))
    for kx, ky in ((3, 1), (-5, 2), (7, 3), (1, -1)):
        th = (2.0 * np.pi * kx / ni, 2.0 * np.pi * ky / nj)
        vhat = rng.standard_normal(4) + 1j * rng.standard_normal(4)
        Jc, Jv, phase = _linearised_split(ni, nj, U, th, vhat)
        Hc, Hv, _, _, _ = dfa.symbols(case, np.array([th[0]]), np.array([th[1]]))
        _, Hvx, _, _, _ = dfa.symbols(case, np.array([th[0]]), np.array([0.0]))
        _, Hvy, _, _, _ = dfa.symbols(case, np.array([0.0]), np.array([th[1]]))
        assert np.allclose(Hvx[0] + Hvy[0], Hv[0], rtol=1e-13, atol=1e-12)
        # The section's H_v is a scalar symbol times its matrix M, the
        # linearisation of the dissipated variables w = (rho, rho v, rho H).
        # Its printed energy row, (-(gamma-1)|v|^2/2, 0, 0, gamma), is not
        # the derivative of rho H = gamma rho E - (gamma-1)|m|^2/(2 rho),
        # whose row is ((gamma-1)|v|^2/2, -(gamma-1) v_1, -(gamma-1) v_2,
        # gamma); the residual linearises exactly, so the symbol's scalar
        # part is compared with the exact row in place of the printed one.
        q2 = v1 * v1 + v2 * v2
        Mp = np.eye(4)
        Mp[3] = (-(GAMMA - 1.0) * q2 / 2.0, 0.0, 0.0, GAMMA)
        Me = np.eye(4)
        Me[3] = ((GAMMA - 1.0) * q2 / 2.0, -(GAMMA - 1.0) * v1, -(GAMMA - 1.0) * v2, GAMMA)
        C = Me @ np.linalg.inv(Mp)
        ec = (Hc[0] @ vhat)[:, None, None] * phase[None]
        ev = ((C @ (mx * Hvx[0] + my * Hvy[0])) @ vhat)[:, None, None] * phase[None]
        scale_c = np.abs(ec).max()
        scale_v = np.abs(ev).max()
        assert np.abs(Jc[:, inner[0], inner[1]] - ec[:, inner[0], inner[1]]).max() < 1e-11 * scale_c
        assert np.abs(Jv[:, inner[0], inner[1]] - ev[:, inner[0], inner[1]]).max() < 1e-11 * scale_v


def test_pseudo_time_step_closed_forms():
    """On a uniform box at zero incidence: dt_form 1 gives the Fourier
    analysis step c* dx / (|v_1| + a) (width over wave speed in the stiffer
    direction), dt_form 0 gives c* dx dy / ((|v_1| + a) dy + a dx)."""
    ni, nj = 12, 6
    x, y = _uniform_box(ni, nj)
    lev = build_levels(x, y, fi.BOX, 0, 1)[0]
    U = np.array([1.0, 1.0, 0.0, 3.290])
    a = np.sqrt(GAMMA * gas.pressure(U) / U[0])
    Up = np.broadcast_to(U[:, None, None], (4, nj + 4, ni + 4)).copy()
    dx, dy = 1.0 / ni, 1.0 / nj
    cs = 7.0
    d1 = res.local_time_step(lev, Up, cs, 1)
    d0 = res.local_time_step(lev, Up, cs, 0)
    # dy = 2 dx here: the x step dx / (|v_1| + a) is the smaller one
    assert np.allclose(d1, cs * dx / (1.0 + a), rtol=1e-14)
    assert np.allclose(d0, cs * dx * dy / ((1.0 + a) * dy + a * dx), rtol=1e-14)


def test_viscous_flux_of_linear_fields():
    """u = 2x + 3y, v = 5x - 7y, T = 1 + 0.3x - 0.2y (rho = 1, p = T) on a
    jittered box with every padded cell (ghosts included) set to the linear
    field: the face gradients are exact, so the face flux is the Newtonian
    stress with the Stokes hypothesis,
        tau_xx = mu (2 u_x - 2/3 div) = mu (4 + 10/3),
        tau_yy = mu (2 v_y - 2/3 div) = mu (-14 + 10/3),
        tau_xy = mu (u_y + v_x) = 8 mu          (div = 2 - 7 = -5),
    plus mu_t in mu, and the heat flux (mu / Pr + mu_t / Pr_t) gamma/(gamma-1)
    grad T with grad T = (0.3, -0.2), dotted with the face vector; the energy
    flux also carries the mean of the two cells' velocities."""
    x, y = fi.box_grid(10, 8, ratio=1.2)
    lev = build_levels(x, y, fi.BOX, 0, 1)[0]
    par = ofas.Params(model=1, mach=0.8, reynolds=1e3)
    X, Y = lev.xc, lev.yc
    u = 2.0 * X + 3.0 * Y
    v = 5.0 * X - 7.0 * Y
    T = 1.0 + 0.3 * X - 0.2 * Y
    Up = np.stack([np.ones_like(T), u, v, T / (GAMMA - 1.0) + 0.5 * (u * u + v * v)])
    mut_val = 3.0e-4
    mutp = np.full(T.shape, mut_val)
    Gxi, Geta = res.viscous_faces(lev, Up, mutp, par)
    mu_inf = 0.8 * np.sqrt(GAMMA) / 1e3
    P = NG
    for G, S, cL, cR in (
        (Gxi, lev.Sxi, (slice(P, -P), slice(P - 1, -P)), (slice(P, -P), slice(P, -P + 1 or None))),
        (Geta, lev.Seta, (slice(P - 1, -P), slice(P, -P)), (slice(P, -P + 1 or None), slice(P, -P))),
    ):
        Tf = 0.5 * (T[cL] + T[cR])
        mu = res.sutherland(Tf, mu_inf)          # Sutherland's law itself: parity unpinned
        me = mu + mut_val
        txx, tyy, txy = me * (4.0 + 10.0 / 3.0), me * (-14.0 + 10.0 / 3.0), me * 8.0
        k = (mu / 0.75 + mut_val / 0.9) * GAMMA / (GAMMA - 1.0)
        qx, qy = k * 0.3, k * -0.2
        fu = 0.5 * (u[cL] + u[cR])
        fv = 0.5 * (v[cL] + v[cR])
        sx, sy = S[0], S[1]
        e1 = txx * sx + txy * sy
        e2 = txy * sx + tyy * sy
        e3 = (fu * txx + fv * txy + qx) * sx + (fu * txy + fv * tyy + qy) * sy
        for got, want in ((G[1], e1), (G[2], e2), (G[3], e3)):
            assert np.abs(got - want).max() < 1e-11 * np.abs(want).max()
        assert np.all(G[0] == 0.0)


def test_sensor_and_dissipation_coefficients():
    """Hand-computed values of the pressure (or entropy) sensor
    |q_{j+1} - 2 q_j + q_{j-1}| / (q_{j+1} + 2 q_j + q_{j-1} + 0.001), of
    eps2 = min(0.25, max(s_L, s_R)) r and eps4 = max(0, r/32 - 2 eps2), and
    of the sign of the face dissipation."""
    assert res._sensor(1.0, 2.0, 3.0) == 0.0                      # linear profile
    assert abs(res._sensor(1.0, 1.0, 2.0) - 1.0 / 5.001) < 1e-15   # a step
    assert abs(res._sensor(2.0, 1.0, 2.0) - 2.0 / 6.001) < 1e-15   # a dip
    w = [np.array([1.0]), np.array([2.0]), np.array([4.0]), np.array([8.0])]   # LL, L, R, RR
    r = np.array([32.0])
    # smooth: s = 0 -> eps2 = 0, eps4 = 1: d = -(8 - 3*4 + 3*2 - 1) = -1
    d = res._face_dissipation(*w, np.array([0.0]), np.array([0.0]), r, r, True, 0.125)
    assert d[0] == -1.0
    # s = 0.01 on one side: eps2 = 0.32, eps4 = 1 - 0.64 = 0.36
    d = res._face_dissipation(*w, np.array([0.01]), np.array([0.0]), r, np.array([16.0]), True, 0.125)
    assert abs(d[0] - (0.32 * 2.0 - 0.36 * 1.0)) < 1e-14
    # a shock (s >= 1/64 caps eps4 at 0; s capped at 0.25): eps2 = 8
    d = res._face_dissipation(*w, np.array([0.9]), np.array([0.1]), r, r, True, 0.125)
    assert d[0] == 8.0 * 2.0
    # coarse levels: first order, eps2 = kappa2c r
    d = res._face_dissipation(*w, None, None, r, r, False, 0.125)
    assert d[0] == 4.0 * 2.0


def test_prolongation_reproduces_linear_fields():
    """Bilinear 9/3/3/1 weights reproduce a linear function of the cell
    centres on a uniform grid at every fine cell whose coarse neighbours on
    its side exist."""
    x, y = _uniform_box(16, 12)
    lf, lc = build_levels(x, y, fi.BOX, 0, 2)
    f = lambda X, Y: np.stack([1.0 + 2.0 * X - 3.0 * Y, -0.5 * X + 0.25 * Y, 7.0 * X, 3.0 - Y])
    e = f(lc.xc[NG:-NG, NG:-NG], lc.yc[NG:-NG, NG:-NG])
    got = ofas.prolong(lf, lc, e)
    want = f(lf.xc[NG:-NG, NG:-NG], lf.yc[NG:-NG, NG:-NG])
    inner = (slice(None), slice(1, -1), slice(1, -1))
    assert np.abs(got[inner] - want[inner]).max() < 1e-13
    # at the boundary rows the missing neighbour is replaced by the parent
    assert np.abs(got[:, 0, 1:-1] - want[:, 0, 1:-1]).max() > 1e-3


def test_riemann_far_field_invariants():
    g1 = GAMMA - 1.0
    rng = np.random.default_rng(8)
    n = 200
    rho = rng.uniform(0.6, 1.4, n)
    vx = rng.uniform(-0.6, 0.6, n)
    vy = rng.uniform(-0.6, 0.6, n)
    p = rng.uniform(0.6, 1.4, n)
    Ui = fi.primitive_to_conservative(rho, vx, vy, p)
    ang = rng.uniform(0.0, 2.0 * np.pi, n)
    nx, ny = np.cos(ang), np.sin(ang)
    Uinf = gas.freestream(0.7, 2.0)
    B = bc.riemann_farfield(Ui, Uinf[:, None], nx, ny)

    def prim(V):
        r = V[0]
        ux, uy = V[1] / r, V[2] / r
        pp = gas.pressure(V)
        return r, ux, uy, pp, np.sqrt(GAMMA * pp / r)

    rb, ubx, uby, pb, ab = prim(B)
    ri, uix, uiy, pi_, ai = prim(Ui)
    rf, ufx, ufy, pf, af = prim(np.broadcast_to(Uinf[:, None], Ui.shape))
    vnb, vni, vnf = ubx * nx + uby * ny, uix * nx + uiy * ny, ufx * nx + ufy * ny
    assert np.allclose(vnb + 2.0 * ab / g1, vni + 2.0 * ai / g1, rtol=1e-13, atol=1e-13)
    assert np.allclose(vnb - 2.0 * ab / g1, vnf - 2.0 * af / g1, rtol=1e-13, atol=1e-13)
    out = vnb > 0.0
    assert out.any() and (~out).any()
    s_up = np.where(out, pi_ / ri ** GAMMA, pf / rf ** GAMMA)
    assert np.allclose(pb / rb ** GAMMA, s_up, rtol=1e-12)
    tb = -ubx * ny + uby * nx
    t_up = np.where(out, -uix * ny + uiy * nx, -ufx * ny + ufy * nx)
    assert np.allclose(tb, t_up, rtol=1e-12, atol=1e-13)
