"""Block SGS preconditioner from the flux-vector-split first-order
linearisation (Section 4.4).

* Eq. "steadylinearized": the upwind linearised operator of cell c is
  Omega_c^-1 sum_f |e_f| (A+_{n_f} u_c + A-_{n_f} u_nb), with the split
  Jacobians evaluated at the arithmetic mean of the two cells' conservative
  states (reading of "the average of the values on both sides") and the
  eigenvalue cutoff of eq. "cutoff".
* Eqs. "d-l-u-matrices-W" / "d-unsteady-W" (additive W, L + D + U =
  I + eta dt* J):
      D_c = (1 + tau eta dt*_c) I + (eta dt*_c / Omega_c) sum_f |S_f| A+_{n_f}
      B_{c,nb} = (eta dt*_c / Omega_c) |S_f| A-_{n_f}
  with tau = 3/(2 dt) for BDF2, 1/dt for the implicit Euler start, 0 steady.
* Eqs. "d-l-u-matrices-J" / "d-unsteady-J" (preconditioned ARK, L + D + U =
  J): the same with the factor 1/Omega_c and diagonal shift tau.
  Readings: n_f is the unit normal pointing out of cell c; couplings to
  boundary ghosts are dropped while D keeps A+ of every face; the wake-cut
  coupling is kept and counts as earlier or later by cell order.
* Eq. "sgs-precon": P = (D+L) D^-1 (D+U), applied by a forward sweep, a
  multiplication by D and a backward sweep (``sgs.c``).

Since A(-n) = -A(n) and |A(-n)| = |A(n)|, the split Jacobians are formed
once per face for the stored face vector (pointing towards +i or +j):
the cell on the low side uses (A+, A-) and the cell on the high side
uses (-A-, -A+).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import gas
from .geometry import NG, CGRID

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libsgs_oracle.so")
        if not os.path.exists(path):
            build()
        _LIB = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        for name in ("sgs_forward", "sgs_backward"):
            f = getattr(_LIB, name)
            f.argtypes = [ctypes.c_int, dp, dp, ip, dp, dp]
            f.restype = None
        f = _LIB.sgs_forward_hyperplane
        f.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ip, dp, dp]
        f.restype = None
    return _LIB


def build():
    """Compile the oracle's C sweep (plain gcc, no contraction of a*b+c)."""
    import subprocess
    src = os.path.join(_HERE, "sgs.c")
    out = os.path.join(_HERE, "libsgs_oracle.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                           "-shared", "-fPIC", src, "-o", out])


def _ptr(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def face_split(lev, Up, d: float):
    """(|S| A+, |S| A-) on every i-face (nj, ni+1, 4, 4) and j-face
    (nj+1, ni, 4, 4), for the stored face vector direction."""
    P = NG
    ni, nj = lev.ni, lev.nj
    out = []
    for (S, UL, UR, W) in (
        (lev.Sxi, Up[:, P:P + nj, P - 1:P + ni], Up[:, P:P + nj, P:P + ni + 1], lev.wxi),
        (lev.Seta, Up[:, P - 1:P + nj, P:P + ni], Up[:, P:P + nj + 1, P:P + ni], lev.weta),
    ):
        ln = np.sqrt(S[0] * S[0] + S[1] * S[1])
        nx = S[0] / ln
        ny = S[1] / ln
        Uf = 0.5 * (UL + UR)
        shift = None
        if W is not None:          # moving mesh: normal grid speed of the face
            shift = (W[0] * S[0] + W[1] * S[1]) / ln
        Ap, Am = gas.split_jacobians(Uf, nx, ny, d, shift)
        out.append((ln[..., None, None] * Ap, ln[..., None, None] * Am))
    return out


def neighbours(lev):
    """Neighbour table (nj*ni, 4) in cell numbering c = j*ni + i."""
    ni, nj = lev.ni, lev.nj
    jj, ii = np.meshgrid(np.arange(nj), np.arange(ni), indexing="ij")
    c = jj * ni + ii
    nb = np.full((nj, ni, 4), -1, dtype=np.int32)
    nb[:, 1:, 0] = c[:, :-1]
    nb[:, :-1, 1] = c[:, 1:]
    nb[1:, :, 2] = c[:-1, :]
    nb[:-1, :, 3] = c[1:, :]
    if lev.topology == CGRID:
        cut = lev.cut_mask()
        partner = ni - 1 - np.arange(ni)
        nb[0, cut, 2] = partner[cut]
    return nb.reshape(nj * ni, 4)


def face_viscous(lev, Up, mutp, par):
    """Scalar thin-layer estimate of the viscous flux Jacobian per face,
    (mu + mu_t)_f (gamma/Pr) |S_f|^2 / (rho_f Omega_f), on every i-face and
    j-face; Omega_f is the mean volume of the two cells."""
    from .residual import sutherland
    P = NG
    ni, nj = lev.ni, lev.nj
    mu_inf = par.mach * np.sqrt(gas.GAMMA) / par.reynolds
    T = gas.pressure(Up) / Up[0]
    out = []
    for (S, cL, cR) in (
        (lev.Sxi, (slice(P, P + nj), slice(P - 1, P + ni)), (slice(P, P + nj), slice(P, P + ni + 1))),
        (lev.Seta, (slice(P - 1, P + nj), slice(P, P + ni)), (slice(P, P + nj + 1), slice(P, P + ni))),
    ):
        rf = 0.5 * (Up[0][cL] + Up[0][cR])
        Tf = 0.5 * (T[cL] + T[cR])
        mue = sutherland(Tf, mu_inf) + 0.5 * (mutp[cL] + mutp[cR])
        s2 = S[0] * S[0] + S[1] * S[1]
        vf = 0.5 * (lev.volp[cL] + lev.volp[cR])
        out.append(((mue * (gas.GAMMA / par.prandtl)) * s2) / (rf * vf))
    return out


class Blocks:
    """D and the four neighbour blocks of every cell, frozen at a state.

    Without ``mutp`` the blocks are the printed ones: the convective
    flux-vector splitting alone.  With ``mutp`` (RANS levels, the
    ``viscous_blocks`` option) a scalar estimate of the viscous Jacobian is
    added: v_f on the diagonal for every face and -v_f on the coupling (both
    then scaled like the convective blocks), v_f from ``face_viscous``.
    This thin-layer term is an extension, not part of the printed formulas:
    on high-Reynolds-number grids with 1e-6 wall spacing it damps the
    laminar sublayer's stiffness, which the convective splitting leaves
    unmatched.
    """

    def __init__(self, lev, Up, dts, par, tau: float = 0.0, aw: bool = True, mutp=None):
        ni, nj = lev.ni, lev.nj
        (Xp, Xm), (Ep, Em) = face_split(lev, Up, par.d_cut)
        if mutp is not None:
            vx, ve = face_viscous(lev, Up, mutp, par)
            eye = np.eye(4)
            Xp = Xp + vx[..., None, None] * eye
            Xm = Xm - vx[..., None, None] * eye
            Ep = Ep + ve[..., None, None] * eye
            Em = Em - ve[..., None, None] * eye
        if aw:
            e = par.eta * dts
            c = e / lev.vol
            diag = 1.0 + tau * e
        else:
            c = 1.0 / lev.vol
            diag = np.full_like(dts, tau)
        acc = ((Xp[:, 1:] - Xm[:, :-1]) + Ep[1:, :]) - Em[:-1, :]
        cc = c[..., None, None]
        D = cc * acc
        for k in range(4):
            D[..., k, k] = D[..., k, k] + diag
        B = np.zeros((nj, ni, 4, 4, 4))
        B[:, :, 0] = -(cc * Xp[:, :-1])     # west: outward normal is -S
        B[:, :, 1] = cc * Xm[:, 1:]         # east
        B[:, :, 2] = -(cc * Ep[:-1, :])     # south (or partner across the cut)
        B[:, :, 3] = cc * Em[1:, :]         # north
        self.ni, self.nj = ni, nj
        self.D = np.ascontiguousarray(D.reshape(nj * ni, 4, 4))
        self.B = np.ascontiguousarray(B.reshape(nj * ni, 4, 4, 4))
        self.nb = np.ascontiguousarray(neighbours(lev))

    # r, y, x as (4, nj, ni) arrays
    def _cells(self, r):
        return np.ascontiguousarray(np.moveaxis(r, 0, -1).reshape(-1, 4))

    def _field(self, v):
        return np.ascontiguousarray(np.moveaxis(v.reshape(self.nj, self.ni, 4), -1, 0))

    def forward(self, r, hyperplane: bool = False):
        rc = self._cells(r)
        y = np.empty_like(rc)
        lib = _lib()
        if hyperplane:
            lib.sgs_forward_hyperplane(self.ni, self.nj, _ptr(self.D), _ptr(self.B),
                                       _ptr(self.nb, ctypes.c_int), _ptr(rc), _ptr(y))
        else:
            lib.sgs_forward(self.ni * self.nj, _ptr(self.D), _ptr(self.B),
                            _ptr(self.nb, ctypes.c_int), _ptr(rc), _ptr(y))
        return self._field(y)

    def backward(self, y):
        yc = self._cells(y)
        x = np.empty_like(yc)
        _lib().sgs_backward(self.ni * self.nj, _ptr(self.D), _ptr(self.B),
                            _ptr(self.nb, ctypes.c_int), _ptr(yc), _ptr(x))
        return self._field(x)

    def apply(self, r):
        """x = P^-1 r."""
        return self.backward(self.forward(r))

    def dense(self):
        """Dense (D+L), D, (D+U) in the cell-major unknown ordering
        (index 4*c + k), for checks on tiny grids."""
        n = self.ni * self.nj
        DL = np.zeros((4 * n, 4 * n))
        DD = np.zeros((4 * n, 4 * n))
        DU = np.zeros((4 * n, 4 * n))
        for c in range(n):
            sl = slice(4 * c, 4 * c + 4)
            DL[sl, sl] = self.D[c]
            DD[sl, sl] = self.D[c]
            DU[sl, sl] = self.D[c]
            for s in range(4):
                m = self.nb[c, s]
                if m < 0:
                    continue
                ms = slice(4 * m, 4 * m + 4)
                if m < c:
                    DL[sl, ms] = self.B[c, s]
                else:
                    DU[sl, ms] = self.B[c, s]
        return DL, DD, DU
