"""Ideal-gas relations, the Euler flux, its normal Jacobian and the flux
vector splitting with the small-eigenvalue cutoff.

Paper: Section 2 (conservative variables, p = (gamma-1) rho (E - |v|^2/2),
H = E + p/rho, gamma = 1.4; the third row of the printed convective flux
repeats the second and is read as rho v_i v_2 + p delta_i2) and Section 4.4
(A = A+ + A-, A+- = (A +- |A|)/2 = R Lambda+- R^-1 at the interface average,
parabolic cutoff of |lambda| below a*d, eq. "cutoff").

All functions broadcast over leading array dimensions.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def pressure(U):
    rho, mx, my, E = U[0], U[1], U[2], U[3]
    return (GAMMA - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)


def freestream(mach: float, alpha_deg: float):
    """Nondimensional free stream: rho = 1, p = 1, a = sqrt(gamma),
    |v| = M sqrt(gamma); this scaling reproduces the paper's physical time
    step 0.486822 (Section 6.4) for M = 0.75, k = 0.202, 36 steps."""
    V = mach * np.sqrt(GAMMA)
    a = alpha_deg * (np.pi / 180.0)
    vx = V * np.cos(a)
    vy = V * np.sin(a)
    E = 1.0 / (GAMMA - 1.0) + 0.5 * (vx * vx + vy * vy)
    return np.array([1.0, vx, vy, E])


def normal_flux(U, p, sx, sy):
    """Convective flux dotted with the (unnormalised) face vector s."""
    rho, mx, my, E = U[0], U[1], U[2], U[3]
    qs = mx * sx + my * sy
    vs = qs / rho
    return np.stack([qs, mx * vs + p * sx, my * vs + p * sy, (E + p) * vs])


def flux_jacobian(U, nx, ny):
    """A_n = d(F . n)/du for unit n, shape (..., 4, 4)."""
    rho = U[0]
    u = U[1] / rho
    v = U[2] / rho
    p = pressure(U)
    H = (U[3] + p) / rho
    g1 = GAMMA - 1.0
    q2 = u * u + v * v
    phi = 0.5 * g1 * q2
    V = u * nx + v * ny
    z = np.zeros_like(rho)
    A = np.empty(rho.shape + (4, 4))
    A[..., 0, :] = np.stack([z, nx + z, ny + z, z], axis=-1)
    A[..., 1, :] = np.stack([phi * nx - u * V, V - (GAMMA - 2.0) * u * nx,
                             u * ny - g1 * v * nx, g1 * nx + z], axis=-1)
    A[..., 2, :] = np.stack([phi * ny - v * V, v * nx - g1 * u * ny,
                             V - (GAMMA - 2.0) * v * ny, g1 * ny + z], axis=-1)
    A[..., 3, :] = np.stack([V * (phi - H), H * nx - g1 * u * V,
                             H * ny - g1 * v * V, GAMMA * V], axis=-1)
    return A


def eigensystem(U, nx, ny):
    """Eigenvalues (V, V, V+a, V-a) and the right / left eigenvector
    matrices R, L = R^-1 of A_n (textbook closed form)."""
    rho = U[0]
    u = U[1] / rho
    v = U[2] / rho
    p = pressure(U)
    a = np.sqrt(GAMMA * p / rho)
    H = (U[3] + p) / rho
    g1 = GAMMA - 1.0
    q2 = u * u + v * v
    V = u * nx + v * ny
    tx, ty = -ny, nx
    Vt = u * tx + v * ty
    one = np.ones_like(rho)
    z = np.zeros_like(rho)
    lam = np.stack([V, V, V + a, V - a], axis=-1)
    R = np.empty(rho.shape + (4, 4))
    R[..., :, 0] = np.stack([one, u, v, 0.5 * q2], axis=-1)
    R[..., :, 1] = np.stack([z, tx + z, ty + z, Vt], axis=-1)
    R[..., :, 2] = np.stack([one, u + a * nx, v + a * ny, H + a * V], axis=-1)
    R[..., :, 3] = np.stack([one, u - a * nx, v - a * ny, H - a * V], axis=-1)
    b = g1 / (a * a)
    L = np.empty(rho.shape + (4, 4))
    L[..., 0, :] = np.stack([1.0 - 0.5 * b * q2, b * u, b * v, -b], axis=-1)
    L[..., 1, :] = np.stack([-Vt, tx + z, ty + z, z], axis=-1)
    L[..., 2, :] = 0.5 * np.stack([0.5 * b * q2 - V / a, nx / a - b * u,
                                   ny / a - b * v, b], axis=-1)
    L[..., 3, :] = 0.5 * np.stack([0.5 * b * q2 + V / a, -nx / a - b * u,
                                   -ny / a - b * v, b], axis=-1)
    return lam, R, L, a


def cutoff_abs(lam, a, d: float):
    """|lambda| with the parabolic cutoff of eq. "cutoff": below a*d it is
    replaced by (a d + lambda^2/(a d))/2 (continuous in value and slope)."""
    al = np.abs(lam)
    if d <= 0.0:
        return al
    ad = a[..., None] * d if np.ndim(lam) > np.ndim(a) else a * d
    return np.where(al <= ad, 0.5 * (ad + al * al / ad), al)


def split_jacobians(U, nx, ny, d: float, shift=None):
    """(A+, A-) = ((A + |A|_c)/2, (A - |A|_c)/2) at state U, unit normal n.
    On a moving face the normal flux is F.n - w_n u, so A and its
    eigenvalues are shifted by the face's normal grid speed ``shift``."""
    A = flux_jacobian(U, nx, ny)
    lam, R, L, a = eigensystem(U, nx, ny)
    if shift is not None:
        A = A - shift[..., None, None] * np.eye(4)
        lam = lam - shift[..., None]
    al = cutoff_abs(lam, a, d)
    absA = np.einsum("...ik,...k,...kj->...ij", R, al, L)
    return 0.5 * (A + absA), 0.5 * (A - absA)
