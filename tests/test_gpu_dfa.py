"""Discrete Fourier analysis on the GPU (fas_dfa through the C ABI) against
the oracle: every pair of phase angles' spectral radius, the amplification
and smoothing factors, the printed amplification factors, sampled pairs of
the aspect-ratio-10000 mesh, and the argument checks (needs a GPU)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dfa as odfa
from oracle import smoother as osm

pytestmark = pytest.mark.gpu

TOL = 1e-10
# With the exact or no preconditioner the iteration matrices of some pairs
# have multiple, defective eigenvalues (G is a multiple of I at zero phase
# and nearly so around it): their moduli are determined only to about the
# square root of the rounding of G, so those cases are compared at 1e-7
TOL_DEFECTIVE = 1e-7


def _tol(precond):
    return TOL if precond == odfa.SGS else TOL_DEFECTIVE
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dfa_amplification_alpha0_ar1.txt")


def _pair(scheme, cstar, d, eta, ar=1.0, u=odfa.U_ALPHA0, unsteady=True, c=200.0, precond=0, unsplit=0,
          mesh=0):
    from paper_1710_04875_amd import fas
    g = fas.DfaCase(u=u, scheme=scheme, cstar=cstar, d=d, eta=eta, ar=ar, c=c, unsteady=int(unsteady),
                    precond=precond, unsplit=unsplit, mesh=mesh)
    o = odfa.DfaCase(u=u, scheme=scheme, cstar=cstar, d=d, eta=eta, ar=ar, c=c, unsteady=unsteady,
                     precond=precond, unsplit=bool(unsplit), mesh=mesh)
    return g, o


CASES = [
    (osm.AW3, 3, 0.5, 0.8, 1.0, odfa.U_ALPHA0, True),
    (osm.PARK3J, 14, 0.5, 0.8, 1.0, odfa.U_ALPHA0, True),
    (osm.AW51, 4, 0.1, 0.6, 4.0, odfa.U_ALPHA45, True),
    (osm.AW52, 30, 0.25, 0.5, 4.0, odfa.U_ALPHA0, False),
    (osm.AW5J, 1e6, 0.5, 0.5, 100.0, odfa.U_ALPHA0, True),
    (osm.PARK51, 2, 0.0, 0.8, 1.0, odfa.U_ALPHA45, True),
    (osm.AW3, 12, 0.1, 0.8, 100.0, odfa.U_ALPHA0, True),
    # exact preconditioner, no preconditioner (unsplit: ERK3), dy = dx / AR
    (osm.AW3, 7, 1.0, 0.8, 1.0, odfa.U_ALPHA0, True, 200.0, odfa.EXACT),
    (osm.PARK3J, 14, 0.5, 0.8, 4.0, odfa.U_ALPHA45, True, 200.0, odfa.EXACT),
    (osm.PARK3J, 0.9, 0.5, 0.8, 1.0, odfa.U_ALPHA0, True, 200.0, odfa.NONE, 1),
    (osm.PARK3J, 0.9, 0.5, 0.8, 4.0, odfa.U_ALPHA0, False, 200.0, odfa.NONE, 0),
    (osm.PARK3J, 900, 0.1, 0.8, 100.0, odfa.U_ALPHA0, True, 200.0, odfa.SGS, 0, odfa.MESH_DX_OVER_AR),
]


def test_every_phase_angle_pair_matches_the_oracle():
    from paper_1710_04875_amd import fas
    pairs = [_pair(*c) for c in CASES]
    amp, smooth, rad = fas.dfa([g for g, _ in pairs], with_radius=True)
    torch.cuda.synchronize()
    rad = rad.cpu().numpy()
    off = 0
    for k, (g, o) in enumerate(pairs):
        a, s, r = odfa.factors(o)
        n = r.size
        got = rad[off:off + n]
        off += n
        tol = _tol(o.precond)
        assert np.abs(got - r).max() <= tol * max(1.0, r.max()), (k, np.abs(got - r).max())
        assert abs(float(amp[k]) - a) <= tol * max(1.0, a), k
        assert abs(float(smooth[k]) - s) <= tol * max(1.0, s), k
        assert float(smooth[k]) <= float(amp[k])
    assert off == rad.size


def test_printed_amplification_factors():
    from paper_1710_04875_amd import fas
    names = {"AW3": osm.AW3, "PARK3J": osm.PARK3J, "AW51": osm.AW51, "AW52": osm.AW52, "AW5J": osm.AW5J}
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                _, s, cs, d, eta, rho = line.split()
                rows.append((names[s], float(cs), float(d), float(eta), float(rho)))
    amp, _ = fas.dfa([fas.DfaCase(scheme=s, cstar=cs, d=d, eta=eta) for s, cs, d, eta, _ in rows])
    amp = amp.cpu().numpy()
    for k, (_, _, _, _, rho) in enumerate(rows):
        assert abs(amp[k] - rho) <= 5e-5, (k, amp[k], rho)


def test_printed_exact_preconditioner_factors():
    from paper_1710_04875_amd import fas
    path = os.path.join(os.path.dirname(__file__), "golden", "dfa_exact_preconditioner_aw3.txt")
    rows = []
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(float(v) for v in line.split()))
    amp, _ = fas.dfa([fas.DfaCase(scheme=osm.AW3, cstar=cs, d=d, eta=0.8, ar=ar, precond=fas.DFA_EXACT)
                      for ar, cs, d, _ in rows])
    amp = amp.cpu().numpy()
    for k, (_, _, _, rho) in enumerate(rows):
        assert abs(amp[k] - rho) <= 5e-5, (k, amp[k], rho)


def test_aspect_ratio_10000_sampled_pairs():
    """The 8 x 80000 mesh at full size: sampled pairs against the oracle,
    one by one, and the factors against the maximum of the radii."""
    from paper_1710_04875_amd import fas
    g, o = _pair(osm.AW3, 1e6, 0.5, 0.8, ar=10000.0)
    amp, smooth, rad = fas.dfa([g], with_radius=True)
    rad = rad.cpu().numpy()
    tx, ty = odfa.phase_angles(o)
    assert rad.size == tx.size == 8 * 80000
    rng = np.random.default_rng(7)
    pick = np.concatenate([rng.choice(tx.size, 200, replace=False), [0, tx.size - 1, int(np.argmax(rad))]])
    G = odfa.iteration_matrices(o, tx[pick], ty[pick])
    ref = np.abs(np.linalg.eigvals(G)).max(axis=1)
    assert np.abs(rad[pick] - ref).max() <= TOL * max(1.0, ref.max())
    assert float(amp[0]) == rad.max()
    hf = np.maximum(np.abs(tx), np.abs(ty)) >= np.pi / 2 - 1e-12
    assert float(smooth[0]) == rad[hf].max()


def test_argument_checks():
    from paper_1710_04875_amd import fas
    for bad in (dict(nx=7), dict(ny=3), dict(u=(0.0, 1.0, 0.0, 3.29)), dict(u=(1.0, 1.0, 0.0, 0.1)),
                dict(cstar=0.0), dict(d=-1.0), dict(ar=0.0), dict(scheme=9), dict(precond=3),
                dict(mesh=2), dict(unsplit=2)):
        with pytest.raises(fas.FasError):
            fas.dfa([fas.DfaCase(**bad)])
