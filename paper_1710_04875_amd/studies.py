"""Convergence studies on the synthetic C-grid family (one GPU).

The analogues of the paper's Section 6 studies on mesh independence and on
the angle of attack, run on the algebraic C-grids of ``fas_inputs`` (the
paper's NACA 64A010 and RAE 2822 meshes are not available).  The family
keeps the wall spacing (1e-6 chord) and the outer boundary (20 chords) and
refines in both directions: 192 x 96, 256 x 128 and 384 x 192 cells (wake
legs of ni / 8).  Grids as short as the paper's (nj = 32) need a wall-normal
growth of more than 2 per cell on this family; every smoother setting
converges poorly or diverges there.

* mesh independence: the steady RANS case on the three grids, AW3, in the
  mode the benchmark uses (d = 0.5, c* = 100 after a ramp) and in the
  paper's robust mode (d = 0.5, c* = 20 for two cycles then 1e4), each set
  solved together as one batch;
* smoothers: AW3 against AW5J, AW51 and AW52 (rate per cycle and per
  second, cost per cycle) and preconditioned ARK3J over c* on the
  256 x 128 case;
* flow angle: alpha = 0, 1, 2, 4 degrees on the 256 x 128 grid, 100 steady
  V-cycles (one batch of four cases) in the benchmark mode and in the
  paper's fast mode (d = 0.05, c* = 100), and the inner iterations of the
  second BDF2 step with dt = 0.486822 after the benchmark-mode cycles.

The rate is the mean residual reduction per V-cycle,
(r_n / r_0)^(1/n).  Usage: python -m paper_1710_04875_amd.studies
"""
from __future__ import annotations

import json
import sys

import numpy as np

MESHES = [(192, 96), (256, 128), (384, 192)]
ANGLES = [0.0, 1.0, 2.0, 4.0]
DT_UNSTEADY = 0.486822


def _rate(h):
    h = np.asarray(h)
    n = len(h) - 1
    return float((h[-1] / h[0]) ** (1.0 / n)) if n > 0 and h[0] > 0 and h[-1] > 0 else float("nan")


def _params(fas, mach, alpha, **kw):
    base = dict(model=fas.FAS_RANS_BL, scheme=fas.FAS_AW3, mach=mach, alpha_deg=alpha, reynolds=1e7,
                n_levels=3, cycle_gamma=1, nu1=1, eta=0.5, d_cut=0.5, cfl=100.0, cfl_ramp=1.0, n_ramp=4,
                ramp_growth=1.5, kappa2c=0.125)
    base.update(kw)
    return fas.Params(**base)


def mesh_independence(cycles=300, drop=6.0, mach=0.8, alpha=0.0, meshes=MESHES):
    """Mean rate per V-cycle of the steady case on the three meshes, for
    the robust (c* = 1e4) and the benchmark (c* = 100) settings."""
    import torch
    import fas_inputs as fi
    from paper_1710_04875_amd import fas
    modes = {"robust_cstar_1e4": dict(cfl=1e4, cfl_ramp=20.0, n_ramp=2, ramp_growth=1e4),
             "bench_cstar_100": dict()}
    out = {}
    for name, kw in modes.items():
        grids, states = [], []
        for ni, nj in meshes:
            x, y = fi.cgrid(ni, nj, ni // 8)
            g = fas.Grid(fi.CGRID, x, y, ni // 8, 3)
            u0 = torch.from_numpy(fi.uniform_state(ni, nj, mach, alpha)).cuda()
            grids.append(g)
            states.append(fas.State(g, _params(fas, mach, alpha, **kw), u0))
        b = fas.Batch(states)
        hist, stat, _ = b.solve(cycles, drop, True)
        torch.cuda.synchronize()
        out[name] = {"%dx%d" % m: {"rate": round(_rate(h), 4), "cycles": len(h) - 1,
                                   "orders": round(float(np.log10(h[0] / np.nanmin(h))), 2), "status": int(s)}
                     for m, h, s in zip(meshes, hist, stat)}
        del b, states, grids
    return out


def flow_angle(cycles=100, mach=0.8, mesh=(256, 128)):
    """Mean rates for alpha = 0, 1, 2, 4: 100 steady V-cycles in the
    benchmark and the fast mode, and the inner cycles of the second BDF2
    step (dt = 0.486822) started from the benchmark-mode steady iterate."""
    import torch
    import fas_inputs as fi
    from paper_1710_04875_amd import fas
    ni, nj = mesh
    x, y = fi.cgrid(ni, nj, ni // 8)
    out = {"mesh": "%dx%d" % mesh}
    for name, kw in (("fast_d_0.05", dict(d_cut=0.05)), ("bench_d_0.5", dict())):
        grids, states = [], []
        for a in ANGLES:
            g = fas.Grid(fi.CGRID, x, y, ni // 8, 3)
            u0 = torch.from_numpy(fi.uniform_state(ni, nj, mach, a)).cuda()
            grids.append(g)
            states.append(fas.State(g, _params(fas, mach, a, **kw), u0))
        b = fas.Batch(states)
        hist, stat, _ = b.solve(cycles, 0.0, True)
        torch.cuda.synchronize()
        del b
        out["steady_" + name] = {
            str(a): {"rate": round(_rate(h), 4), "orders": round(float(np.log10(h[0] / np.nanmin(h))), 2),
                     "status": int(s)} for a, h, s in zip(ANGLES, hist, stat)}
    unsteady = {}
    for a, st in zip(ANGLES, states):
        st.dual_time_step(DT_UNSTEADY, a, cycles, 0.0)
        h, s = st.dual_time_step(DT_UNSTEADY, a, cycles, 0.0)
        unsteady[str(a)] = {"rate": round(_rate(h), 4), "orders": round(float(np.log10(h[0] / np.nanmin(h))), 2),
                            "status": int(s)}
    out["unsteady_second_step_bench"] = unsteady
    return out


def smoother_comparison(cap=600, drop=6.0, park_cstars=(0.25, 0.5, 1.0, 2.0, 4.0)):
    """The relative comparisons of Section 6 (the steady columns of the
    tables of smoother rates and times) on the 256 x 128 workload: AW3,
    AW5J, AW51 and AW52 at the benchmark setting (d = 0.5, eta = 0.5,
    c* = 100 after the ramp, V-cycles), each to a 6-order drop: cycles,
    seconds, rate per cycle and per second, and the cost of a cycle relative
    to AW3; and preconditioned ARK3J over a range of c*, where the paper
    finds it unstable above c* = 1."""
    import time
    import torch
    import fas_inputs as fi
    from paper_1710_04875_amd import fas
    case = fi.steady_cgrid_case()
    x, y = case.grid()
    g = fas.Grid(case.topology, x, y, case.n_wake, 3)
    u0 = torch.from_numpy(case.initial_state(x, y)).cuda()
    out = {"workload": "steady RANS 256x128 C-grid (the benchmark case), V-cycles, 6-order drop"}
    schemes = (("AW3", fas.FAS_AW3), ("AW5J", fas.FAS_AW5J), ("AW51", fas.FAS_AW51), ("AW52", fas.FAS_AW52))
    for name, sc in schemes:
        st = fas.State(g, _params(fas, case.mach, case.alpha_deg, scheme=sc), u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, s = st.cycle(cap, drop)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        n = len(h) - 1
        r = _rate(h)
        out[name] = {"status": int(s), "cycles": n, "seconds": round(t, 4), "ms_per_cycle": round(1e3 * t / n, 4),
                     "rate_per_cycle": round(r, 4),
                     "rate_per_second": float("%.4g" % (r ** (n / t))) if np.isfinite(r) else None,
                     "orders": round(float(np.log10(h[0] / np.nanmin(h))), 2)}
    base = out["AW3"]["ms_per_cycle"]
    for name, _ in schemes:
        out[name]["cycle_cost_vs_aw3"] = round(out[name]["ms_per_cycle"] / base, 3)
    park = {}
    for cs in park_cstars:
        st = fas.State(g, _params(fas, case.mach, case.alpha_deg, scheme=fas.FAS_PARK3J, cfl=cs, cfl_ramp=min(cs, 1.0)),
                       u0)
        h, s = st.cycle(300, drop)
        park[str(cs)] = {"status": int(s), "cycles": len(h) - 1, "rate_per_cycle": round(_rate(h), 4),
                         "orders": round(float(np.log10(h[0] / np.nanmin(h))), 2)}
    out["PARK3J_by_cstar"] = park
    return out


def main():
    res = {"mesh_independence": mesh_independence(), "flow_angle": flow_angle(),
           "smoother_comparison": smoother_comparison()}
    json.dump(res, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main()
