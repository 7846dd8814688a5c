"""Discrete Fourier analysis of the preconditioned smoothers (Section
"Discrete Fourier Analysis"): the iteration matrix of one AW or
preconditioned ARK iteration for the linearised Euler equations with the JST
discretisation on a periodic Cartesian mesh, block-diagonalised by the
discrete Fourier transform into one 4x4 complex matrix per pair of phase
angles, and its amplification and smoothing factors.

Oracle: test infrastructure.  Only tests, the smoke check and the benchmark's
CPU baseline use it; it shares no code with the HIP path.

The operators follow the section's subsections:
* JST: H = H_c + H_v.  H_c = (A (E_x - E_x^-1) dy + B (E_y - E_y^-1) dx) /
  (2 dx dy), plus 3/(2 dt) I in the unsteady case; H_v = M [eps2 second
  differences + eps4 fourth differences] / (dx dy), with the matrix M of the
  section (differences of rho H expressed through rho and rho E);
* SGS: L = -(f / Omega)(dy A+ E_x^-1 + dx B+ E_y^-1), U = (f / Omega)(dy A-
  E_x + dx B- E_y), D = (f / Omega)(dy (A+ - A-) + dx (B+ - B-)) plus 3/(2 dt)
  I (preconditioned ARK, eqs. "d-l-u-matrices-J", "d-unsteady-J", f = 1) or
  plus (1 + 3 eta dt* / (2 dt)) I (additive W, eqs. "d-l-u-matrices-W",
  "d-unsteady-W", f = eta dt*); A+- from the cutoff splitting (eq. "cutoff");
  P = (D + L) D^-1 (D + U) (eq. "sgs-precon");
* the low-storage stages of Section 4 applied to one Fourier mode:
  U_0 = I, V_0 = P^-1 H_v, U_i = I - alpha_i dt* (P^-1 H_c U_{i-1} + V_{i-1}),
  V_i = beta_{i+1} P^-1 H_v U_i + (1 - beta_{i+1}) V_{i-1}; G = U_s.
Shift operators become E_x = exp(i Theta_x), E_y = exp(i Theta_y).

Preconditioners: the SGS factorisation above, the exact first-order
operator P = D + L + U (the tables' "exact precond." columns: W = I +
eta dt* J with J the flux-split linearisation, or P = J), or none (P = I,
the explicit schemes of Table "ERK-ARK"); with every beta set to 1 the
additive schemes become the unsplit ERK / W forms.

Readings (the text leaves these open; they reproduce the printed AR = 1
amplification factors of the ARK3J, AW3 and AW5 tables at alpha = 0 to all
four printed digits, and the exact-preconditioner AW3 factors at AR 1
(d = 0, 0.1, 0.25 and 1), 100 and 10000 (d = 0 and 0.1)):
* mesh: nx = 8 cells of width 1/8 in x, dy = AR dx, ny = 8 AR; phase angles
  2 pi k / n for k = -n/2 + 1 .. n/2 (the alternative dy = dx / AR, the
  8 AR cells filling the unit height, is an option; it fits fewer printed
  values);
* steps: dt* = c* min(dx / (|v_1| + a), dy / (|v_2| + a)) and dt with c in
  place of c*: the smaller directional CFL step, which is dx / (|v_1| + a)
  for every printed case of the default mesh;
* JST coefficients: the pressure sensor of the constant state is zero, so
  eps2 = 0 and eps4 = r / 32 per direction, r = |v_k| + a;
* the amplification factor is the largest spectral radius over every pair of
  phase angles; the smoothing factor takes the pairs with max(|Theta_x|,
  |Theta_y|) >= pi/2.  Parity unpinned for the smoothing factor: the printed
  smoothing factors are smaller than the spectral radius of every high
  frequency mode of these symbols, and in two rows of the exact-preconditioner
  ARK3J columns the printed smoothing factor exceeds the printed
  amplification factor, which no maximum over a subset of the modes gives,
  so the paper's definition differs in a way the text does not state.

Not reproduced with these readings (nor with dy = dx / AR, a step from
either width or speed, or the identity in the steady ARK diagonal): Table
"ERK-ARK" (the explicit three-stage schemes are unstable at c* = 0.9, where
the printed factor 0.9933 is exactly G at Theta = 0), the
exact-preconditioner ARK3J columns, and the SGS columns at AR 100 and
10000 beyond d = 0.1 (AW3 within 1.2e-3 up to d = 0.1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .gas import GAMMA, flux_jacobian, pressure, split_jacobians
from .smoother import SCHEMES

# the section's two linearisation states (Mach 0.8 at 45 and at 0 degrees)
U_ALPHA45 = (1.0, np.sqrt(2.0) / 2.0, np.sqrt(2.0) / 2.0, 3.290)
U_ALPHA0 = (1.0, 1.0, 0.0, 3.290)


SGS, EXACT, NONE = 0, 1, 2       # preconditioner of the stages
MESH_AR_DX, MESH_DX_OVER_AR = 0, 1


@dataclass
class DfaCase:
    u: tuple = U_ALPHA0     # linearisation state (rho, rho v1, rho v2, rho E)
    scheme: int = 0         # smoother.AW3 ... (coefficients and W or P ~ J)
    cstar: float = 3.0      # pseudo CFL c*
    d: float = 0.5          # eigenvalue cutoff
    eta: float = 0.8        # W parameter (additive W schemes)
    ar: float = 1.0         # aspect ratio (the mesh reading below)
    c: float = 200.0        # physical CFL
    nx: int = 8
    unsteady: bool = True
    precond: int = SGS      # SGS, EXACT (P = D + L + U) or NONE (P = I)
    unsplit: bool = False   # every beta = 1 (the ERK / unsplit W forms)
    mesh: int = MESH_AR_DX  # dy = AR dx, or dy = dx / AR

    @property
    def ny(self) -> int:
        return int(round(self.nx * self.ar))


def _state(U):
    U = np.asarray(U, dtype=np.float64)
    rho = U[0]
    v1, v2 = U[1] / rho, U[2] / rho
    a = np.sqrt(GAMMA * pressure(U) / rho)
    return U, v1, v2, a


def steps(case: DfaCase):
    """(dx, dy, dt*, dt) of the reading above."""
    _, v1, v2, a = _state(case.u)
    dx = 1.0 / case.nx
    dy = dx / case.ar if case.mesh == MESH_DX_OVER_AR else case.ar * dx
    base = min(dx / (abs(v1) + a), dy / (abs(v2) + a))
    return dx, dy, case.cstar * base, case.c * base


def coefficients(case: DfaCase):
    """(alpha, beta, W form) of the case's scheme (beta = 1 if unsplit)."""
    alpha, beta, wform = SCHEMES[case.scheme]
    if case.unsplit:
        beta = tuple(1.0 for _ in beta)
    return alpha, beta, wform


def _preconditioner(case, L, D, Uu):
    if case.precond == EXACT:
        return D + L + Uu
    if case.precond == NONE:
        return np.broadcast_to(np.eye(4, dtype=complex), D.shape).copy()
    return (D + L) @ np.linalg.solve(D, D + Uu)


def phase_angles(case: DfaCase):
    """All (Theta_x, Theta_y) pairs of the nx x ny mesh, Theta_x slowest."""
    kx = np.arange(-case.nx // 2 + 1, case.nx // 2 + 1)
    ky = np.arange(-case.ny // 2 + 1, case.ny // 2 + 1)
    tx = 2.0 * np.pi * kx / case.nx
    ty = 2.0 * np.pi * ky / case.ny
    TX, TY = np.meshgrid(tx, ty, indexing="ij")
    return TX.ravel(), TY.ravel()


def symbols(case: DfaCase, tx, ty):
    """Fourier symbols (H_c, H_v, L, D, U), each (n, 4, 4) complex."""
    U, v1, v2, a = _state(case.u)
    dx, dy, dts, dt = steps(case)
    vol = dx * dy
    _, beta_unused, wform = coefficients(case)
    A = flux_jacobian(U, 1.0, 0.0)
    B = flux_jacobian(U, 0.0, 1.0)
    Ap, Am = split_jacobians(U, 1.0, 0.0, case.d)
    Bp, Bm = split_jacobians(U, 0.0, 1.0, case.d)
    ex = np.exp(1j * np.asarray(tx))[:, None, None]
    ey = np.exp(1j * np.asarray(ty))[:, None, None]
    I4 = np.eye(4)
    Hc = (A * (ex - 1.0 / ex) * dy + B * (ey - 1.0 / ey) * dx) / (2.0 * vol)
    if case.unsteady:
        Hc = Hc + (1.5 / dt) * I4
    M = np.eye(4)
    M[3, 0] = -(GAMMA - 1.0) * (v1 * v1 + v2 * v2) / 2.0
    M[3, 3] = GAMMA
    e4x, e4y = (abs(v1) + a) / 32.0, (abs(v2) + a) / 32.0
    fourth_x = ex * ex - 4.0 * ex + 6.0 - 4.0 / ex + 1.0 / (ex * ex)
    fourth_y = ey * ey - 4.0 * ey + 6.0 - 4.0 / ey + 1.0 / (ey * ey)
    Hv = M * (e4x * fourth_x * dy + e4y * fourth_y * dx) / vol
    f = case.eta * dts if wform else 1.0
    L = -(f / vol) * (dy * Ap / ex + dx * Bp / ey)
    Uu = (f / vol) * (dy * Am * ex + dx * Bm * ey)
    D = (f / vol) * (dy * (Ap - Am) + dx * (Bp - Bm)) * np.ones_like(ex)
    if wform:
        D = D + (1.0 + (1.5 * case.eta * dts / dt if case.unsteady else 0.0)) * I4
    elif case.unsteady:
        D = D + (1.5 / dt) * I4
    return Hc, Hv, L, D, Uu


def iteration_matrices(case: DfaCase, tx, ty):
    """G (n, 4, 4) of one smoother iteration per pair of phase angles."""
    alpha, beta, _ = coefficients(case)
    _, _, dts, _ = steps(case)
    Hc, Hv, L, D, Uu = symbols(case, tx, ty)
    P = _preconditioner(case, L, D, Uu)
    Hcb = np.linalg.solve(P, Hc)
    Hvb = np.linalg.solve(P, Hv)
    I4 = np.broadcast_to(np.eye(4, dtype=complex), Hc.shape)
    Ui, V = I4, Hvb
    s = len(alpha)
    for i in range(s):
        Ui = I4 - alpha[i] * dts * (Hcb @ Ui + V)
        if i + 1 < s:
            V = beta[i + 1] * (Hvb @ Ui) + (1.0 - beta[i + 1]) * V
    return Ui


def factors(case: DfaCase):
    """(amplification factor, smoothing factor, spectral radius per pair of
    phase angles in the order of phase_angles)."""
    tx, ty = phase_angles(case)
    G = iteration_matrices(case, tx, ty)
    rad = np.abs(np.linalg.eigvals(G)).max(axis=1)
    hf = np.maximum(np.abs(tx), np.abs(ty)) >= np.pi / 2.0 - 1e-12
    return float(rad.max()), float(rad[hf].max()), rad


def full_iteration_matrix(case: DfaCase):
    """The same iteration assembled on the whole periodic nx x ny mesh as
    dense 4N x 4N matrices (no Fourier transform): cell (i, j) at block
    4 (i ny + j), shifts as periodic block permutations."""
    U, v1, v2, a = _state(case.u)
    dx, dy, dts, dt = steps(case)
    vol = dx * dy
    alpha, beta, wform = coefficients(case)
    nx, ny = case.nx, case.ny
    N = nx * ny
    A = flux_jacobian(U, 1.0, 0.0)
    B = flux_jacobian(U, 0.0, 1.0)
    Ap, Am = split_jacobians(U, 1.0, 0.0, case.d)
    Bp, Bm = split_jacobians(U, 0.0, 1.0, case.d)

    def shift(di, dj):
        # (E u)_{i,j} = u_{i+di, j+dj}
        S = np.zeros((N, N))
        for i in range(nx):
            for j in range(ny):
                S[i * ny + j, ((i + di) % nx) * ny + (j + dj) % ny] = 1.0
        return S

    def blk(S, X):
        return np.kron(S, X)

    Ex, Exm, Ey, Eym = shift(1, 0), shift(-1, 0), shift(0, 1), shift(0, -1)
    Ex2, Exm2, Ey2, Eym2 = shift(2, 0), shift(-2, 0), shift(0, 2), shift(0, -2)
    I = np.eye(4 * N)
    Hc = (blk(Ex - Exm, A) * dy + blk(Ey - Eym, B) * dx) / (2.0 * vol)
    if case.unsteady:
        Hc = Hc + (1.5 / dt) * I
    M = np.eye(4)
    M[3, 0] = -(GAMMA - 1.0) * (v1 * v1 + v2 * v2) / 2.0
    M[3, 3] = GAMMA
    IN = np.eye(N)
    fx = Ex2 - 4.0 * Ex + 6.0 * IN - 4.0 * Exm + Exm2
    fy = Ey2 - 4.0 * Ey + 6.0 * IN - 4.0 * Eym + Eym2
    Hv = blk((abs(v1) + a) / 32.0 * fx * dy + (abs(v2) + a) / 32.0 * fy * dx, M) / vol
    f = case.eta * dts if wform else 1.0
    L = -(f / vol) * (blk(Exm, Ap) * dy + blk(Eym, Bp) * dx)
    Uu = (f / vol) * (blk(Ex, Am) * dy + blk(Ey, Bm) * dx)
    D = (f / vol) * blk(IN, dy * (Ap - Am) + dx * (Bp - Bm))
    if wform:
        D = D + (1.0 + (1.5 * case.eta * dts / dt if case.unsteady else 0.0)) * I
    elif case.unsteady:
        D = D + (1.5 / dt) * I
    if case.precond == EXACT:
        P = D + L + Uu
    elif case.precond == NONE:
        P = np.eye(4 * N)
    else:
        P = (D + L) @ np.linalg.solve(D, D + Uu)
    Hcb = np.linalg.solve(P, Hc)
    Hvb = np.linalg.solve(P, Hv)
    Ui, V = I, Hvb
    s = len(alpha)
    for i in range(s):
        Ui = I - alpha[i] * dts * (Hcb @ Ui + V)
        if i + 1 < s:
            V = beta[i + 1] * (Hvb @ Ui) + (1.0 - beta[i + 1]) * V
    return Ui
