"""The allocation-free Fourier analysis entry point against fas_dfa,
through the C ABI, on two calls in a row (the second with fewer cases and
smaller meshes), and its size limit (needs a GPU)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dfa as odfa
from oracle import smoother as osm

pytestmark = pytest.mark.gpu


def _cases(big):
    from paper_1710_04875_amd import fas
    out = [fas.DfaCase(scheme=osm.AW3, cstar=3, d=0.5, eta=0.8),
           fas.DfaCase(scheme=osm.PARK3J, cstar=14, d=0.5, ar=4.0, u=odfa.U_ALPHA45),
           fas.DfaCase(scheme=osm.AW3, cstar=7, d=1.0, precond=fas.DFA_EXACT)]
    if big:
        out += [fas.DfaCase(scheme=osm.AW51, cstar=4, d=0.1, eta=0.6, ar=100.0),
                fas.DfaCase(scheme=osm.AW5J, cstar=1e6, d=0.5, eta=0.5, ar=100.0, unsteady=0),
                fas.DfaCase(scheme=osm.PARK3J, cstar=0.9, precond=fas.DFA_NONE, unsplit=1)]
    return out


def _run(entry, cases):
    from paper_1710_04875_amd import fas
    lib = fas.load()
    arr = (fas._DfaCase * len(cases))(*[c.c_struct() for c in cases])
    dev = torch.device("cuda", torch.cuda.current_device())
    amp = torch.full((len(cases),), -1.0, dtype=torch.float64, device=dev)
    smooth = torch.full_like(amp, -1.0)
    total = sum(int(a.nx) * int(a.ny) for a in arr)
    rad = torch.full((total,), -1.0, dtype=torch.float64, device=dev)
    st = getattr(lib, entry)(arr, len(cases), ctypes.c_void_p(amp.data_ptr()), ctypes.c_void_p(smooth.data_ptr()),
                             ctypes.c_void_p(rad.data_ptr()),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == fas.FAS_OK, lib.fas_last_error()
    torch.cuda.synchronize()
    return amp.cpu().numpy(), smooth.cpu().numpy(), rad.cpu().numpy()


def test_noalloc_equals_fas_dfa_on_two_calls():
    for big in (True, False):
        cases = _cases(big)
        ref = _run("fas_dfa", cases)
        got = _run("fas_dfa_noalloc", cases)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        # and the oracle, pair by pair (the bar of the other analysis tests)
        off = 0
        for k, c in enumerate(cases):
            o = odfa.DfaCase(u=c.u, scheme=c.scheme, cstar=c.cstar, d=c.d, eta=c.eta, ar=c.ar, c=c.c,
                             unsteady=bool(c.unsteady), precond=c.precond, unsplit=bool(c.unsplit), mesh=c.mesh)
            a, s, r = odfa.factors(o)
            n = r.size
            # 1e-10 (1e-7 where the exact or no preconditioner gives
            # defective eigenvalues, as in the other analysis tests)
            tol = 1e-10 if c.precond == 0 else 1e-7
            assert np.abs(got[2][off:off + n] - r).max() <= tol * max(1.0, r.max()), k
            off += n


def test_noalloc_rejects_more_cases_than_its_table():
    from paper_1710_04875_amd import fas
    lib = fas.load()
    n = 1025
    arr = (fas._DfaCase * n)(*[fas.DfaCase().c_struct() for _ in range(n)])
    dev = torch.device("cuda", torch.cuda.current_device())
    amp = torch.empty(n, dtype=torch.float64, device=dev)
    st = lib.fas_dfa_noalloc(arr, n, ctypes.c_void_p(amp.data_ptr()), ctypes.c_void_p(amp.data_ptr()), None,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == fas.FAS_EINVAL
