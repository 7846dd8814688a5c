"""Discrete adjoint of the steady fine-level residual (test infrastructure).

Everything here is differentiated by the complex step: F(u + i h e)
carries h dF/du e in its imaginary part to rounding accuracy, so the dense
Jacobian and the parameter derivatives below are exact derivatives of the
oracle's own discrete residual, not finite-difference approximations.

Readings (the paper states no adjoint):
* the functional is the lift (and drag) coefficient of the pressure force
  on the solid wall, with the wall pressure the residual itself uses (the
  mean of the wall cell and its ghost), force = -sum p_w S over the wall
  faces (S points into the fluid), q_inf = rho_inf |v_inf|^2 / 2, chord 1;
* the eddy viscosity is frozen at the state (frozen-turbulence adjoint):
  the Baldwin-Lomax field is evaluated once at the real state and is not
  differentiated;
* the adjoint equation is (dF/du)^T lambda = -dJ/du and the gradient of J
  with respect to a flow parameter q is dJ/dq = dJ/dq|_u + lambda^T dF/dq.

* grid-node sensitivities differentiate the fine level's metrics (face
  vectors, mean face vectors, volumes, centres, ghost reflections) with
  respect to the node coordinates; the eddy viscosity stays frozen, so the
  wall distance of the turbulence model is not differentiated.

Vector layout: component-major flattening of (4, nj, ni) arrays; node
arrays are (nj + 1, ni + 1), i fastest.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import gas
from .bc import fill_ghosts
from .geometry import NG, Level
from .residual import baldwin_lomax, padded_eddy_viscosity, split_residual

H_CS = 1.0e-30


def _padded(S, u, uinf):
    lev = S.levels[0]
    Up = np.zeros((4, lev.nj + 2 * NG, lev.ni + 2 * NG), dtype=np.result_type(u, uinf))
    Up[:, NG:NG + lev.nj, NG:NG + lev.ni] = u
    fill_ghosts(Up, lev, uinf, noslip=S.par.model == 1)
    return Up


def frozen_mut(S, u):
    """Padded eddy viscosity at the (real) state u, or None for Euler."""
    if S.par.model != 1:
        return None
    lev = S.levels[0]
    return padded_eddy_viscosity(lev, baldwin_lomax(lev, _padded(S, u, S.uinf), S.par))


def fine_residual(S, u, mutp, mach=None, alpha_deg=None):
    """Steady fine-level F(u) (no forcing, no time term) with the frozen eddy
    viscosity mutp; u, mach and alpha may be complex."""
    mach = S.par.mach if mach is None else mach
    alpha_deg = S.par.alpha_deg if alpha_deg is None else alpha_deg
    par = dataclasses.replace(S.par, mach=mach, alpha_deg=alpha_deg)
    uinf = gas.freestream(mach, alpha_deg)
    Up = _padded(S, u, uinf)
    Fc, Fv = split_residual(S.levels[0], Up, par, True, mutp, None, None)
    return Fc + Fv


def _fine_level(S, x, y):
    L0 = S.levels[0]
    return Level(x, y, L0.topology, L0.n_wake)


def residual_at_nodes(S, u, mutp, x, y):
    """Steady fine-level F(u) on the grid with nodes (x, y) (which may be
    complex), frozen eddy viscosity mutp."""
    lev = _fine_level(S, x, y)
    Up = np.zeros((4, lev.nj + 2 * NG, lev.ni + 2 * NG), dtype=np.result_type(u, lev.x, S.uinf))
    Up[:, NG:NG + lev.nj, NG:NG + lev.ni] = u
    fill_ghosts(Up, lev, S.uinf, noslip=S.par.model == 1)
    Fc, Fv = split_residual(lev, Up, S.par, True, mutp, None, None)
    return Fc + Fv


def residual_node_jvp(S, u, mutp, vx, vy):
    """(dF/dx) vx + (dF/dy) vy at fixed u: the derivative of the residual
    along the node displacement (vx, vy), by the complex step."""
    L0 = S.levels[0]
    return residual_at_nodes(S, u, mutp, L0.x + 1j * H_CS * vx, L0.y + 1j * H_CS * vy).imag / H_CS


def forces(S, u, mach=None, alpha_deg=None, nodes=None):
    """(C_L, C_D) of the wall pressure force of state u (on the grid with
    nodes = (x, y) if given, which may be complex)."""
    mach = S.par.mach if mach is None else mach
    alpha_deg = S.par.alpha_deg if alpha_deg is None else alpha_deg
    lev = S.levels[0] if nodes is None else _fine_level(S, *nodes)
    uinf = gas.freestream(mach, alpha_deg)
    Up = np.zeros((4, lev.nj + 2 * NG, lev.ni + 2 * NG), dtype=np.result_type(u, lev.x, uinf))
    Up[:, NG:NG + lev.nj, NG:NG + lev.ni] = u
    fill_ghosts(Up, lev, uinf, noslip=S.par.model == 1)
    p = gas.pressure(Up)
    cols = slice(NG, NG + lev.ni)
    pw = 0.5 * (p[NG - 1, cols] + p[NG, cols])
    wall = ~lev.cut_mask()
    fx = -np.sum((pw * lev.Seta[0][0])[wall])
    fy = -np.sum((pw * lev.Seta[1][0])[wall])
    a = alpha_deg * (np.pi / 180.0)
    q = 0.5 * (mach * mach * gas.GAMMA)
    cl = (fy * np.cos(a) - fx * np.sin(a)) / q
    cd = (fx * np.cos(a) + fy * np.sin(a)) / q
    return cl, cd


def residual_node_vjp(S, u, mutp, lam):
    """((dF/dx)^T lam, (dF/dy)^T lam) on the node arrays, one complex-step
    residual per node coordinate (small grids only)."""
    L0 = S.levels[0]
    out = []
    for axis in (0, 1):
        g = np.empty(L0.x.shape)
        for J in range(L0.x.shape[0]):
            for I in range(L0.x.shape[1]):
                e = np.zeros(L0.x.shape)
                e[J, I] = 1.0
                z = np.zeros(L0.x.shape)
                jv = residual_node_jvp(S, u, mutp, e if axis == 0 else z, z if axis == 0 else e)
                g[J, I] = np.sum(lam * jv)
        out.append(g)
    return out[0], out[1]


def lift_node_jvp(S, u, vx, vy):
    """dC_L/dx . vx + dC_L/dy . vy at fixed u (complex step)."""
    L0 = S.levels[0]
    return forces(S, u, nodes=(L0.x + 1j * H_CS * vx, L0.y + 1j * H_CS * vy))[0].imag / H_CS


def lift_node_derivative(S, u, vx, vy, lam=None):
    """Total derivative of C_L of the converged state u along the node
    displacement (vx, vy): dC_L/dX v + lam . (dF/dX v), with lam the dense
    adjoint solution of (dF/du)^T lam = -dC_L/du (computed if not given)."""
    mutp = frozen_mut(S, u)
    if lam is None:
        _, lam = lift_gradient(S, u)
    return lift_node_jvp(S, u, vx, vy) + np.sum(lam * residual_node_jvp(S, u, mutp, vx, vy))


def dense_jacobian(S, u, mutp):
    """dF/du (4N x 4N) at u, column by column."""
    n = u.size
    J = np.empty((n, n))
    flat = u.reshape(-1)
    for k in range(n):
        uc = flat.astype(complex)
        uc[k] += 1j * H_CS
        J[:, k] = fine_residual(S, uc.reshape(u.shape), mutp).imag.reshape(-1) / H_CS
    return J


def residual_param_partials(S, u, mutp):
    """(dF/dalpha_deg, dF/dmach) at fixed u, as (4, nj, ni) arrays."""
    da = fine_residual(S, u, mutp, alpha_deg=S.par.alpha_deg + 1j * H_CS).imag / H_CS
    dm = fine_residual(S, u, mutp, mach=S.par.mach + 1j * H_CS).imag / H_CS
    return da, dm


def lift_partials(S, u):
    """(dC_L/du as (4, nj, ni), dC_L/dalpha_deg, dC_L/dmach) at fixed u."""
    flat = u.reshape(-1)
    g = np.empty(flat.size)
    for k in range(flat.size):
        uc = flat.astype(complex)
        uc[k] += 1j * H_CS
        g[k] = forces(S, uc.reshape(u.shape))[0].imag / H_CS
    da = forces(S, u, alpha_deg=S.par.alpha_deg + 1j * H_CS)[0].imag / H_CS
    dm = forces(S, u, mach=S.par.mach + 1j * H_CS)[0].imag / H_CS
    return g.reshape(u.shape), da, dm


def lift_gradient(S, u):
    """dC_L/d(alpha_deg, mach) at a converged state u by the dense adjoint."""
    mutp = frozen_mut(S, u)
    J = dense_jacobian(S, u, mutp)
    g, cla, clm = lift_partials(S, u)
    lam = np.linalg.solve(J.T, -g.reshape(-1))
    da, dm = residual_param_partials(S, u, mutp)
    return (cla + lam @ da.reshape(-1), clm + lam @ dm.reshape(-1)), lam.reshape(u.shape)


def smoother_map(S, u, frozen):
    """One fine-level smoother iteration (Section 4: the low-storage stages
    with the split f^c / f^v of Section 4.1) from the state u, which may be
    complex, with dt*, the SGS blocks and the eddy viscosity held at the
    values ``frozen`` = S.prepare(0) computed at the real starting state."""
    from .smoother import additive_iteration
    _, dts, mutp, blocks = frozen
    lev = S.levels[0]

    def split(v):
        Up = _padded(S, v, S.uinf)
        return split_residual(lev, Up, S.par, True, mutp, None, None)

    def apply(r):   # P^-1 is linear with real blocks
        if np.iscomplexobj(r):
            return blocks.apply(np.ascontiguousarray(r.real)) + 1j * blocks.apply(np.ascontiguousarray(r.imag))
        return blocks.apply(r)

    if S.aw:
        inc = lambda r: apply(dts * r)
    else:
        inc = lambda r: dts * apply(r)
    return additive_iteration(u, split, inc, S.alpha, S.beta)


def smoother_jacobian(S, u):
    """dS/du (4N x 4N, component-major flattening) of the smoother map at
    the steady state u with its frozen quantities, column by column by the
    complex step."""
    S.set_u(0, u)
    frozen = S.prepare(0)
    n = u.size
    J = np.empty((n, n))
    flat = u.reshape(-1)
    for k in range(n):
        uc = flat.astype(complex)
        uc[k] += 1j * H_CS
        J[:, k] = smoother_map(S, uc.reshape(u.shape), frozen).imag.reshape(-1) / H_CS
    return J


# ------------------------------------------------- dual time stepping
# Eq. "nonlin-eq" with the start of Section 6: step n solves
#   F(u^n; alpha_n, M) + T^n = 0,  T^1 = (u^1 - u^0)/dt,
#   T^n = (3 u^n - 4 u^{n-1} + u^{n-2})/(2 dt) (n >= 2),
# from the steady solution u^0 of F(u; alpha_0, M) = 0.  The functional is
# the time-averaged lift J = (1/N) sum_{n=1..N} C_L(u^n, alpha_n).

def unsteady_states(S, dt, alphas, max_cycles, drop):
    """u^0 .. u^N of the oracle's dual time stepping from its current
    (converged, steady) state, the far-field angle set to alphas[n] at step n."""
    states = [S.u(0)]
    for n in range(1, len(alphas)):
        S.begin_time_step(dt, alphas[n])
        S.run_cycles(max_cycles, drop)
        states.append(S.u(0))
    return states


def _jacobian_at(S, u, mutp, alpha):
    n = u.size
    J = np.empty((n, n))
    flat = u.reshape(-1)
    for k in range(n):
        uc = flat.astype(complex)
        uc[k] += 1j * H_CS
        J[:, k] = fine_residual(S, uc.reshape(u.shape), mutp, alpha_deg=alpha).imag.reshape(-1) / H_CS
    return J


def _lift_grad_u(S, u, alpha):
    flat = u.reshape(-1)
    g = np.empty(flat.size)
    for k in range(flat.size):
        uc = flat.astype(complex)
        uc[k] += 1j * H_CS
        g[k] = forces(S, uc.reshape(u.shape), alpha_deg=alpha)[0].imag / H_CS
    return g


def unsteady_direct_gradient(S, states, dt, alphas):
    """(J, dJ/dM, dJ/dalpha_n per degree for n = 0..N) by forward
    (direct) sensitivities through the steps: for a parameter q,
    v^0 = -F_u^-1 F_q at the steady start, and for n >= 1
    (F_u + tau_n I) v^n = -F_q - dT^n/du^{n-1} v^{n-1} - dT^n/du^{n-2} v^{n-2},
    dJ/dq = (1/N) sum_n (dC_L/du . v^n + dC_L/dq).  Dense Jacobians by the
    complex step (small grids only), the eddy viscosity frozen at each
    state.  Independent of any transposed (adjoint) product."""
    N = len(states) - 1
    w = 1.0 / N
    mach = S.par.mach
    nu = states[0].size
    Jn, Fa, Fm, g, cla, clm, cl = [], [], [], [], [], [], []
    for n, u in enumerate(states):
        a = alphas[n]
        uinf = gas.freestream(mach, a)
        mutp = None
        if S.par.model == 1:
            lev = S.levels[0]
            mutp = padded_eddy_viscosity(lev, baldwin_lomax(lev, _padded(S, u, uinf),
                                                            dataclasses.replace(S.par, alpha_deg=a)))
        Jn.append(_jacobian_at(S, u, mutp, a))
        Fa.append((fine_residual(S, u, mutp, alpha_deg=a + 1j * H_CS).imag / H_CS).reshape(-1))
        Fm.append((fine_residual(S, u, mutp, mach=mach + 1j * H_CS, alpha_deg=a).imag / H_CS).reshape(-1))
        g.append(_lift_grad_u(S, u, a))
        cla.append(forces(S, u, alpha_deg=a + 1j * H_CS)[0].imag / H_CS)
        clm.append(forces(S, u, mach=mach + 1j * H_CS, alpha_deg=a)[0].imag / H_CS)
        cl.append(forces(S, u, alpha_deg=a)[0])
    I = np.eye(nu)

    def sensitivity(Fq):
        # Fq[n]: dF_n/dq (zero vector where q does not enter step n)
        v = [np.linalg.solve(Jn[0], -Fq[0])]
        for n in range(1, N + 1):
            tau = 1.0 / dt if n == 1 else 1.5 / dt
            rhs = -Fq[n]
            if n == 1:
                rhs = rhs + v[0] / dt                     # dT^1/du^0 = -1/dt
            else:
                rhs = rhs + (2.0 / dt) * v[n - 1] - (0.5 / dt) * v[n - 2]
            v.append(np.linalg.solve(Jn[n] + tau * I, rhs))
        return v

    z = np.zeros(nu)
    vm = sensitivity(Fm)
    dJ_dm = w * sum(g[n] @ vm[n] + clm[n] for n in range(1, N + 1))
    dJ_da = []
    for k in range(N + 1):
        va = sensitivity([Fa[n] if n == k else z for n in range(N + 1)])
        dJ_da.append(w * sum(g[n] @ va[n] + (cla[n] if n == k else 0.0) for n in range(1, N + 1)))
    J = w * sum(cl[1:])
    return J, dJ_dm, np.array(dJ_da)
