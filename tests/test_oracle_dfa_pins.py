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


@pytest.mark.parametrize("case", [
    dfa.DfaCase(scheme=sm.AW3, cstar=3, d=0.5),
    dfa.DfaCase(scheme=sm.PARK3J, cstar=14, d=0.5),
    dfa.DfaCase(u=dfa.U_ALPHA45, scheme=sm.AW51, cstar=5, d=0.1, eta=0.6),
    dfa.DfaCase(scheme=sm.AW3, cstar=40, d=0.25, ar=2.0, unsteady=False),
], ids=["aw3", "park3j", "aw51-45deg", "aw3-steady-ar2"])
def test_fourier_blocks_are_the_spectrum_of_the_periodic_operator(case):
    """Brute force: the dense 4N x 4N iteration matrix of the periodic mesh
    (explicit shift permutations, no transform) has exactly the union of the
    4x4 symbols' eigenvalues."""
    G = dfa.full_iteration_matrix(case)
    full = np.sort(np.abs(np.linalg.eigvals(G)))
    tx, ty = dfa.phase_angles(case)
    blocks = np.sort(np.abs(np.linalg.eigvals(dfa.iteration_matrices(case, tx, ty))).ravel())
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
