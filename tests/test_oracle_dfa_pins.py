"""Pins of the discrete Fourier analysis oracle: the amplification factors
the paper prints (aspect ratio 1, alpha = 0), the spectrum of the whole
periodic iteration matrix assembled without the Fourier transform, and the
symmetries of the symbols."""
import os

import numpy as np
import pytest

from oracle import dfa
from oracle import smoother as sm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dfa_amplification_alpha0_ar1.txt")
GOLDEN_EXACT = os.path.join(os.path.dirname(__file__), "golden", "dfa_exact_preconditioner_aw3.txt")
SCHEME = {"AW3": sm.AW3, "PARK3J": sm.PARK3J, "AW51": sm.AW51, "AW52": sm.AW52, "AW5J": sm.AW5J}


def _golden():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                t, s, cs, d, eta, rho = line.split()
                rows.append((t, s, float(cs), float(d), float(eta), float(rho)))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: "%s-%s-c%g-d%g-eta%g" % r[:5])
def test_printed_amplification_factors(row):
    """The four printed digits (half a unit of the last digit)."""
    _, s, cs, d, eta, rho = row
    case = dfa.DfaCase(u=dfa.U_ALPHA0, scheme=SCHEME[s], cstar=cs, d=d, eta=eta, ar=1.0)
    amp, _, _ = dfa.factors(case)
    assert abs(amp - rho) <= 5e-5, (amp, rho)


def _golden_exact():
    rows = []
    with open(GOLDEN_EXACT) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                ar, cs, d, rho = (float(v) for v in line.split())
                rows.append((ar, cs, d, rho))
    return rows


@pytest.mark.parametrize("row", _golden_exact(), ids=lambda r: "ar%g-c%g-d%g" % r[:3])
def test_printed_exact_preconditioner_factors(row):
    """The exact-preconditioner AW3 columns: four printed digits."""
    ar, cs, d, rho = row
    case = dfa.DfaCase(u=dfa.U_ALPHA0, scheme=sm.AW3, cstar=cs, d=d, eta=0.8, ar=ar, precond=dfa.EXACT)
    tx, ty = dfa.phase_angles(case)
    # the AR 10000 mesh has 640000 pairs: chunks keep the dense solves small
    amp = max(float(np.abs(np.linalg.eigvals(dfa.iteration_matrices(case, tx[k:k + 65536],
                                                                     ty[k:k + 65536]))).max())
              for k in range(0, tx.size, 65536))
    assert abs(amp - rho) <= 5e-5, (amp, rho)


def test_exact_preconditioner_at_zero_phase_is_the_stability_polynomial():
    """Closed form: with P = D + L + U every shift is 1 at Theta = 0, so
    J(0) holds only the BDF2 term and W(0) = (1 + 3 eta dt*/(2 dt)) I; the
    iteration is the three-stage polynomial 1 + z + a3 a2 z^2 + a3 a2 a1 z^3
    of z = -dt* (3/(2 dt)) / (1 + 3 eta dt*/(2 dt))."""
    case = dfa.DfaCase(scheme=sm.AW3, cstar=3, d=0.25, eta=0.8, precond=dfa.EXACT)
    _, _, dts, dt = dfa.steps(case)
    q = 1.5 * dts / dt
    z = -q / (1.0 + 0.8 * q)
    a1, a2, a3 = sm.SCHEMES[sm.AW3][0]
    g = 1.0 + z + a3 * a2 * z * z + a3 * a2 * a1 * z ** 3
    G0 = dfa.iteration_matrices(case, np.array([0.0]), np.array([0.0]))[0]
    assert np.abs(G0 - g * np.eye(4)).max() < 1e-14
    # without a preconditioner the unsplit scheme is the same polynomial of
    # z = -dt* 3/(2 dt) at Theta = 0
    ex = dfa.DfaCase(scheme=sm.PARK3J, cstar=0.9, precond=dfa.NONE, unsplit=True)
    _, _, dts, dt = dfa.steps(ex)
    z = -1.5 * dts / dt
    g = 1.0 + z + a3 * a2 * z * z + a3 * a2 * a1 * z ** 3
    G0 = dfa.iteration_matrices(ex, np.array([0.0]), np.array([0.0]))[0]
    assert np.abs(G0 - g * np.eye(4)).max() < 1e-14
    assert abs(g - 0.9933) < 5e-5       # the printed value of Table "ERK-ARK"


@pytest.mark.parametrize("case", [
    dfa.DfaCase(scheme=sm.AW3, cstar=3, d=0.5),
    dfa.DfaCase(scheme=sm.PARK3J, cstar=14, d=0.5),
    dfa.DfaCase(u=dfa.U_ALPHA45, scheme=sm.AW51, cstar=5, d=0.1, eta=0.6),
    dfa.DfaCase(scheme=sm.AW3, cstar=40, d=0.25, ar=2.0, unsteady=False),
    dfa.DfaCase(scheme=sm.AW3, cstar=7, d=1.0, precond=dfa.EXACT),
    dfa.DfaCase(scheme=sm.PARK3J, cstar=0.5, d=0.5, precond=dfa.NONE, unsplit=True),
    dfa.DfaCase(scheme=sm.PARK3J, cstar=20, d=0.5, ar=2.0, mesh=dfa.MESH_DX_OVER_AR),
], ids=["aw3", "park3j", "aw51-45deg", "aw3-steady-ar2", "aw3-exact", "erk3", "park3j-dx-over-ar"])
def test_fourier_blocks_are_the_spectrum_of_the_periodic_operator(case):
    """Brute force: the dense 4N x 4N iteration matrix of the periodic mesh
    (explicit shift permutations, no transform) has exactly the union of the
    4x4 symbols' eigenvalues."""
    G = dfa.full_iteration_matrix(case)
    tx, ty = dfa.phase_angles(case)
    Gb = dfa.iteration_matrices(case, tx, ty)
    # the dense matrix maps every Fourier mode v exp(i (Theta_x i + Theta_y j))
    # to (G(Theta) v) exp(...): an exact property, no eigenvalue conditioning
    nx, ny = case.nx, case.ny
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    rng = np.random.default_rng(2)
    for m in rng.choice(tx.size, 6, replace=False):
        ph = np.exp(1j * (tx[m] * ii + ty[m] * jj)).ravel()
        v = rng.standard_normal(4) + 1j * rng.standard_normal(4)
        w = np.kron(ph, v)
        want = np.kron(ph, Gb[m] @ v)
        assert np.abs(G @ w - want).max() < 1e-12 * max(1.0, np.abs(want).max())
    if case.precond == dfa.SGS:
        # and the spectra agree (the SGS blocks have simple eigenvalues here;
        # the unpreconditioned and exact ones have multiple, defective ones,
        # which eigenvalue routines resolve only to about sqrt(rounding))
        full = np.sort(np.abs(np.linalg.eigvals(G)))
        blocks = np.sort(np.abs(np.linalg.eigvals(Gb)).ravel())
        assert full.shape == blocks.shape
        assert np.abs(full - blocks).max() < 1e-11


def test_symbol_symmetries_and_limits():
    case = dfa.DfaCase(scheme=sm.AW3, cstar=3, d=0.5, ar=4.0)
    tx, ty = dfa.phase_angles(case)
    G = dfa.iteration_matrices(case, tx, ty)
    Gm = dfa.iteration_matrices(case, -tx, -ty)
    # real base matrices: the symbol at -Theta is the conjugate one
    assert np.abs(Gm - np.conj(G)).max() < 1e-12
    # steady, Theta = 0: H = 0 and every stage leaves the mode unchanged
    st = dfa.DfaCase(scheme=sm.PARK3J, cstar=10, d=0.5, unsteady=False)
    G0 = dfa.iteration_matrices(st, np.array([0.0]), np.array([0.0]))[0]
    assert np.abs(G0 - np.eye(4)).max() < 1e-12
    # c* -> 0: no pseudo-time step, G -> I on every mode
    tiny = dfa.DfaCase(scheme=sm.AW3, cstar=1e-9, d=0.5)
    Gt = dfa.iteration_matrices(tiny, *dfa.phase_angles(tiny))
    assert np.abs(Gt - np.eye(4)).max() < 1e-6
    # the smoothing factor never exceeds the amplification factor
    amp, smf, rad = dfa.factors(case)
    assert smf <= amp and rad.shape == tx.shape
