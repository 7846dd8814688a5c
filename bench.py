#!/usr/bin/env python3
"""Benchmark: AW3 + SGS FAS V-cycles on the steady RANS C-grid (one GPU).

Workload: 256 x 128 algebraic C-grid around a 10 %-thick symmetric NACA
4-digit section (wall spacing 1e-6 chord), Re = 1e7, M = 0.8, angle of
attack drawn from U[0, 2] deg (seed 3), Baldwin-Lomax RANS, FAS V-cycle on
3 levels, AW3 smoother with the SGS preconditioner built from the printed
convective blocks (d = 0.5, eta = 0.5, c* = 100 after a start-up ramp from
c* = 1; the c* = 1e4 robust mode stalls at two orders on this grid).  A step
is one FAS cycle including the residual-norm evaluation and stopping test
(the library replays a captured graph per cycle); the kernel breakdown and
the sweep's launch duration come from as many cycles again, launched
directly with HIP events around each launch.  value = fine cells x cycles
/ s ("fine-cell cycles/s": one fine-level AW3 iteration per V-cycle), FP64
residual, FP64 preconditioner.  Also reported: the same with the FP32
preconditioner, the time to a 6-order residual drop for both, both block
forms in V- and W-cycles, the 64 x 64 Euler box on a single grid, the
roofline of the dominant kernel, and the CPU oracle on every host core on
a bounded sample of the same workload.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per cell of one SGS launch (forward + backward
# sweep of one stage, FP64, blocks recomputed): 144 + 144
SWEEP_BYTES_PER_CELL = 288.0
# one residual evaluation per stage: u 32 + geometry 40 + f 32 + blended
# accumulator 2 x 32 on average (440 B over three stages)
RESIDUAL_BYTES_PER_CELL = 440.0 / 3.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def workload_params(fas, fp32=False):
    import fas_inputs as fi
    case = fi.steady_cgrid_case()
    p = fas.Params(model=fas.FAS_RANS_BL, scheme=fas.FAS_AW3, mach=case.mach,
                   alpha_deg=case.alpha_deg, reynolds=case.reynolds, n_levels=3,
                   cycle_gamma=1, nu1=1, eta=0.5, d_cut=0.5, cfl=100.0, cfl_ramp=1.0,
                   n_ramp=4, ramp_growth=1.5, kappa2c=0.125, precond_fp32=1 if fp32 else 0,
                   viscous_blocks=0, dt_form=1)
    return case, p


def level_cells(ni, nj, levels):
    return [(ni >> l) * (nj >> l) for l in range(levels)]


def run_gpu(fas, torch, steps, warmup, fp32, drop_cap):
    case, p = workload_params(fas, fp32)
    x, y = case.grid()
    u0 = torch.from_numpy(case.initial_state(x, y)).cuda()
    g = fas.Grid(case.topology, x, y, case.n_wake, p.n_levels)
    out = {}
    # throughput: warmup cycles, then K timed cycles (replayed from the
    # library's captured cycle graph)
    st = fas.State(g, p, u0)
    st.cycle(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, status = st.cycle(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    # kernel timing: K more cycles launched directly with HIP events around
    # every launch of the timed kernel classes, on the library's stream (the
    # events cost about a tenth of the cycle time, so the throughput region
    # runs without them)
    st.profile(True)
    hp, _ = st.cycle(steps)
    torch.cuda.synchronize()
    prof = st.profile_read()
    st.profile(False)
    out["prof_cycles"] = len(hp) - 1
    n = len(hist) - 1
    N = case.ni * case.nj
    out["ms_per_step"] = 1e3 * t / max(n, 1)
    out["value"] = N * n / t
    out["steps_done"] = n
    out["prof"] = prof
    out["status"] = status
    if getattr(run_gpu, "no_drop", False):
        out["drop"] = None
        out["deep"] = None
        out["final_state"] = st.get_state().cpu().numpy()
        out["case"] = case
        out["params"] = p
        return out
    # time to a 6-order drop from the initial state
    st2 = fas.State(g, p, u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h2, status2 = st2.cycle(drop_cap, 6.0)
    torch.cuda.synchronize()
    t2 = time.perf_counter() - t0
    drop = math.log10(h2[0] / h2.min()) if len(h2) > 1 and h2.min() > 0 else 0.0
    reached = bool(len(h2) > 1 and h2[-1] <= h2[0] * 1e-6)
    out["drop"] = {"reached": reached, "seconds": t2 if reached else None,
                   "cycles": len(h2) - 1, "orders_reached": round(drop, 3),
                   "seconds_run": round(t2, 4),
                   "avg_rate": round(float((h2[-1] / h2[0]) ** (1.0 / max(len(h2) - 1, 1))), 4)}
    out["final_state"] = st2.get_state().cpu().numpy()
    # the same solve continued to a 10-order drop (converged solutions of
    # the two preconditioner precisions are compared there)
    h3, _ = st2.cycle(1500, 10.0 - drop if reached else 4.0)
    out["deep"] = {"orders": round(float(drop + math.log10(h3[0] / h3.min())), 2),
                   "cycles": out["drop"]["cycles"] + len(h3) - 1}
    out["deep_state"] = st2.get_state().cpu().numpy()
    out["case"] = case
    out["params"] = p
    return out


def block_forms_section(fas, torch, cap):
    """The preconditioner's two block forms on the 256 x 128 workload (the
    printed convective blocks and the thin-layer viscous term) in the
    V-cycle of the workload and in the paper's W-cycle: cycles, time and
    rate to a 6-order drop from the initial state."""
    import fas_inputs as fi
    case, _ = workload_params(fas)
    x, y = case.grid()
    u0 = torch.from_numpy(case.initial_state(x, y)).cuda()
    g = fas.Grid(case.topology, x, y, case.n_wake, 3)
    out = {}
    for vb in (0, 1):
        for gamma in (1, 2):
            _, p = workload_params(fas)
            p.viscous_blocks, p.cycle_gamma = vb, gamma
            st = fas.State(g, p, u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h, status = st.cycle(cap, 6.0)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            n = len(h) - 1
            out["%s_%s" % ("viscous_blocks" if vb else "printed_blocks", "W" if gamma == 2 else "V")] = {
                "reached": bool(status == fas.FAS_OK), "cycles": n, "seconds": round(t, 4),
                "ms_per_cycle": round(1e3 * t / max(n, 1), 4),
                "orders": round(float(math.log10(h[0] / h.min())), 3),
                "avg_rate": round(float((h[-1] / h[0]) ** (1.0 / max(n, 1))), 4)}
    return out


def box_section(fas, torch, iters=50):
    """Config C1: the 64 x 64 jittered Euler box (wall-side stretching 1.1),
    single grid, 50 AW3 iterations with the SGS preconditioner from the
    bump-and-noise state, in the paper's robust mode (eta 0.5, d 0.5, c* 1e4
    after two iterations at 20) and fast mode (d 0.05, c* 100): cell-iters/s
    of the single-grid solve (each iteration with its residual-norm check,
    replayed from the library's captured graph) and the residual drop."""
    import numpy as np
    import fas_inputs as fi
    x, y = fi.box_grid(64, 64)
    u0 = torch.from_numpy(fi.box_initial_state(x, y)).cuda()
    g = fas.Grid(fi.BOX, x, y, 0, 1)
    out = {"workload": "Euler 64x64 jittered box, single grid, %d AW3+SGS iterations" % iters}
    for mode, kw in (("robust", dict(d_cut=0.5, cfl=1.0e4, cfl_ramp=20.0, n_ramp=2)),
                     ("fast", dict(d_cut=0.05, cfl=100.0, cfl_ramp=20.0, n_ramp=2))):
        p = fas.Params(model=fas.FAS_EULER, scheme=fas.FAS_AW3, mach=0.8, alpha_deg=0.0, n_levels=1, eta=0.5, **kw)
        st = fas.State(g, p, u0)
        st.cycle(iters)                     # warm-up
        st.set_state(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, status = st.cycle(iters)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        n = len(h) - 1
        out[mode] = {"cell_iters_per_s": round(64 * 64 * n / (ms * 1e-3), 1),
                     "ms_per_iteration": round(ms / n, 4), "iterations": n, "status": int(status),
                     "orders": round(float(math.log10(h[0] / np.nanmin(h))), 3),
                     "avg_rate": round(float((h[-1] / h[0]) ** (1.0 / n)), 4) if np.isfinite(h[-1]) else None}
    return out


def sweep_roofline(res, case, levels):
    ms, cnt = res["prof"]["sweep"]
    cells = level_cells(case.ni, case.nj, levels)
    # per cycle one AW3 iteration on every level: 3 sweep launches per level
    per_cycle = 3.0 * sum(cells) * SWEEP_BYTES_PER_CELL
    cycles = res["prof_cycles"]
    achieved = per_cycle * cycles / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
            "kernel": "k_sgs4 (forward + backward hyperplane block-SGS sweep, one launch per stage)",
            "avg_launch_us": round(1e3 * ms / max(cnt, 1), 3), "launches": cnt,
            "launch_timing": "HIP events around each sweep launch on the library stream, over %d cycles "
                             "launched directly after the timed ones" % cycles,
            "algorithmic_bytes_per_cell": SWEEP_BYTES_PER_CELL}


def sweep_source_hash():
    """Hash of the sources that define the sweep kernel and the
    configuration it is launched in: the internal header, and the SGS-sweep
    and sweep-configuration sections of fas_kernels.hip."""
    csrc = os.path.join(ROOT, "paper_1710_04875_amd", "csrc")
    with open(os.path.join(csrc, "fas_kernels.hip")) as f:
        k = f.read()
    a = k.index("// ------------------------------------------------------------- SGS sweeps")
    b = k.index("// ------------------------------------------------------------ transfers")
    c = k.index("// Sweep configurations:")
    d = k.index("void launch_sgs(", c)
    h = hashlib.sha256()
    with open(os.path.join(csrc, "fas_internal.h"), "rb") as f:
        h.update(f.read())
    h.update(k[a:b].encode())
    h.update(k[c:d].encode())
    return h.hexdigest()[:16]


def load_traffic(kernel_key):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    calibrated) if the committed counter summary matches these sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel_key)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernels_sha") != sweep_source_hash():
        return None
    return d.get("bytes_per_launch")


def traffic_summary(fetch_dir, write_dir, calf_dir, calw_dir):
    """Calibrated HBM bytes per sweep launch from four rocprofv3 counter
    runs of this file: FETCH_SIZE and WRITE_SIZE over the sweep kernels of the
    throughput workload, and the same counters over --calibrate-copy (a
    256 MiB device copy, which reads and writes 262144 KiB per dispatch).
    Writes profiles/traffic_k_sgs_c2_fp64.json and prints the per-level
    table."""
    import csv
    import numpy as np

    def rows(d):
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            return list(csv.DictReader(f))

    def per_kernel(d):
        g = {}
        for r in rows(d):
            g.setdefault((r["Kernel_Name"], int(r["Grid_Size"])), []).append(float(r["Counter_Value"]))
        return {k: float(np.mean(v)) for k, v in g.items()}

    copy_kib = 262144.0
    calf = max(v for (n, _), v in per_kernel(calf_dir).items() if "copyBuffer" in n)
    calw = max(v for (n, _), v in per_kernel(calw_dir).items() if "copyBuffer" in n)
    ff, fw = copy_kib / calf, copy_kib / calw
    fetch, write = per_kernel(fetch_dir), per_kernel(write_dir)
    cells = level_cells(256, 128, 3)
    keys = sorted((k for k in fetch if "k_sgs" in k[0]), key=lambda k: -fetch[k])
    assert len(keys) == 3, keys
    lines, per = [], []
    for k, c in zip(keys, cells):
        b = (fetch[k] * ff + write[k] * fw) * 1024.0
        per.append(b)
        lines.append("| %d cells | `%s` (grid %d) | %.1f | %.1f | %.4g | %.4g | %.2f |" % (
            c, k[0].replace("void ", "").replace("fas::(anonymous namespace)::", "").split("(")[0], k[1],
            fetch[k], write[k], b, c * SWEEP_BYTES_PER_CELL, b / (c * SWEEP_BYTES_PER_CELL)))
    out = {"kernel": "k_sgs4 (FP64)", "workload": "256x128 RANS C-grid V-cycle",
           "kernels_sha": sweep_source_hash(), "bytes_per_launch": round(float(np.mean(per)), 1),
           "fetch_factor": ff, "write_factor": fw,
           "source": "profiles/k_sgs4_c2_rans_256x128_hbm_traffic.md"}
    with open(os.path.join(ROOT, "profiles", "traffic_k_sgs_c2_fp64.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("calibration: FETCH %.1f KiB (x%.4f), WRITE %.1f KiB (x%.4f) per 262144 KiB copy" % (calf, ff, calw, fw))
    print("| level | kernel | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | calibrated bytes/launch | "
          "algorithmic bytes/launch | ratio |")
    print("|---|---|---|---|---|---|---|")
    print("\n".join(lines))
    print("mean over the levels: %.4g bytes per launch" % out["bytes_per_launch"])


# FP64 operations per pair of phase angles of the Fourier analysis that do
# not depend on the data (a complex multiply-add is 8, a division 11): the
# solve D^-1 (D + U) (786), the product P = (D + L) X (512), the solve with
# eight right-hand columns (1346), per stage a product and update (608,
# s stages and s - 1 blends), the Hessenberg reduction (400); the shifted QR
# iterations come on top, so this is a lower bound
def dfa_flops_per_pair(stages):
    """FP64 operations per pair that do not depend on the data: D, D + L and
    D + U (484), D^-1 (D + U) with the real D (262), (D + L) D^-1 (D + U)
    (480), the right-hand sides H_c and H_v (180), the 8-column complex
    solve (1132), the Householder reduction to Hessenberg form (720) and per
    product of the stage recursion 580 (2 s - 1 of them).  The split
    Jacobians, the trigonometric functions and the QR sweeps are left out,
    so the count is a lower bound."""
    return 484 + 262 + 480 + 180 + 1132 + 720 + 580 * (2 * stages - 1)


def dfa_section(fas, torch):
    """Discrete Fourier analysis over the paper's table grid: schemes ARK3J,
    AW3, AW51, AW52, AW5J x cutoffs d = 0, 0.1, 0.25, 0.5, 1 x aspect ratios
    1, 100, 10000 (8 x 8 AR phase angles) x c* = 3, 30, 1e3, 1e6, Mach 0.8,
    alpha 0, c = 200: one fas_dfa call over all of it, timed with HIP events
    on the library's stream (median of three after a warm-up call); the
    printed amplification factors at aspect ratio 1 as a check; the oracle on
    a bounded sample as the CPU baseline."""
    import numpy as np
    from oracle import dfa as odfa
    stages = {fas.FAS_PARK3J: 3, fas.FAS_AW3: 3, fas.FAS_AW51: 5, fas.FAS_AW52: 5, fas.FAS_AW5J: 5}
    cases = [fas.DfaCase(scheme=sc, cstar=cs, d=d, ar=ar) for sc in stages for d in (0.0, 0.1, 0.25, 0.5, 1.0)
             for ar in (1.0, 100.0, 10000.0) for cs in (3.0, 30.0, 1e3, 1e6)]
    pairs = [c.nx * int(round(c.nx * c.ar)) for c in cases]
    fas.dfa(cases)
    torch.cuda.synchronize()
    runs = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        amp, smooth = fas.dfa(cases)
        e1.record()
        torch.cuda.synchronize()
        runs.append(e0.elapsed_time(e1))
    ms = sorted(runs)[1]
    flops = float(sum(p * dfa_flops_per_pair(stages[c.scheme]) for p, c in zip(pairs, cases)))
    ach = flops / (ms * 1e-3) / 1e12
    # the printed amplification factors (aspect ratio 1, alpha 0)
    printed = [(fas.FAS_PARK3J, 1, 0.0, 0.8, 0.9974), (fas.FAS_PARK3J, 14, 0.5, 0.8, 0.9722),
               (fas.FAS_AW3, 3, 0.5, 0.8, 0.9841), (fas.FAS_AW3, 7, 1.0, 0.8, 0.9765),
               (fas.FAS_AW51, 4, 0.5, 0.5, 0.9776), (fas.FAS_AW5J, 3, 0.1, 0.5, 0.9815)]
    pa, _ = fas.dfa([fas.DfaCase(scheme=sc, cstar=cs, d=d, eta=eta) for sc, cs, d, eta, _ in printed])
    dev = float(np.max(np.abs(pa.cpu().numpy() - np.array([r[-1] for r in printed]))))
    # CPU baseline: the oracle on the aspect-ratio-100 cases of the first scheme
    sample = [c for c in cases if c.ar == 100.0][:20]
    t0 = time.perf_counter()
    npairs = 0
    for c in sample:
        o = odfa.DfaCase(u=c.u, scheme=c.scheme, cstar=c.cstar, d=c.d, eta=c.eta, ar=c.ar, c=c.c)
        npairs += odfa.factors(o)[2].size
        if time.perf_counter() - t0 > 15.0:
            break
    tc = time.perf_counter() - t0
    return {"cases": len(cases), "pairs": int(sum(pairs)), "ms": round(ms, 3),
            "pairs_per_s": round(sum(pairs) / (ms * 1e-3), 1),
            "max_dev_printed_amplification": dev,
            "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": 78.6, "unit": "TFLOP/s",
                         "frac": round(ach / 78.6, 5), "traffic": None,
                         "kernel": "k_dfa (one thread per pair of phase angles)",
                         "flops": "lower bound: %d FP64 operations per pair for 3 stages, %d for 5" % (
                             dfa_flops_per_pair(3), dfa_flops_per_pair(5))},
            "cpu_baseline": {"value": round(npairs / tc, 1), "unit": "pairs/s", "cores": 1, "kind": "oracle",
                             "sample": "%d pairs of the aspect-ratio-100 cases (numpy, vectorised)" % npairs}}


# concurrent case groups of the batched solves (fas_batch_create)
BATCH_GROUPS = 2


def batch_params(fas, c, fp32, vblk=1):
    # the batch's tall grids need the thin-layer viscous block term (the
    # printed blocks diverge on the 512 x 128 and 1024 x 256 grids)
    return fas.Params(model=fas.FAS_RANS_BL, scheme=fas.FAS_AW3, mach=c.mach, alpha_deg=c.alpha_deg,
                      reynolds=c.reynolds, n_levels=3, cycle_gamma=1, nu1=1, eta=0.5, d_cut=0.5,
                      cfl=100.0, cfl_ramp=1.0, n_ramp=4, ramp_growth=1.5, kappa2c=0.125,
                      precond_fp32=1 if fp32 else 0, viscous_blocks=vblk, dt_form=0)


def batch_section(fas, torch, cap, loop_cycles, full_loop):
    """64 steady RANS cases on uneven C-grids (128..512 x 64..256, seed 4):
    the batched engine (one launch per kernel over all cases, one captured
    graph per cycle) to a 6-order drop per case with the FP32 and the FP64
    preconditioner, and the FP64 per-case loop (the same kernels, one case
    after another)."""
    import numpy as np
    import fas_inputs as fi
    cases = fi.batch_cases(64, seed=4)
    cells = np.array([c.ni * c.nj for c in cases], dtype=np.float64)
    grids = []
    for c in cases:
        x, y = c.grid()
        grids.append((fas.Grid(c.topology, x, y, c.n_wake, 3), torch.from_numpy(c.initial_state(x, y)).cuda()))
    out = {"cases": len(cases), "fine_cells": int(cells.sum()), "cycle_cap": cap, "groups": BATCH_GROUPS}
    finals, cycles, status = {}, {}, {}
    # the headline runs use concurrent case groups; the one-group runs give
    # the batched kernels' own timing (a group's launch covers fewer cases)
    for fp32, groups in ((True, BATCH_GROUPS), (False, BATCH_GROUPS), (True, 1), (False, 1)):
        tag = ("fp32_precond" if fp32 else "fp64") + ("" if groups == BATCH_GROUPS else "_one_group")
        log("batch %s: create + autotune" % tag)
        sts = [fas.State(g, batch_params(fas, c, fp32), u0) for (g, u0), c in zip(grids, cases)]
        b = fas.Batch(sts, autotune=True, groups=groups)
        torch.cuda.synchronize()
        log("batch %s: solve to 6 orders (graph)" % tag)
        t0 = time.perf_counter()
        hist, stat, _ = b.solve(cap, 6.0, True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        nd = np.array([len(h) - 1 for h in hist])
        conv = stat == 0
        finals[tag] = [st.get_state().cpu().numpy() for st in sts]
        cycles[tag] = nd
        status[tag] = stat
        r = {"seconds": round(t, 3), "converged": int(conv.sum()),
             "diverged": int((stat == -4).sum()),
             "cycles_total": int(nd.sum()), "cycles_max": int(nd.max()),
             "cell_cycles_per_s": round(float((cells * nd).sum() / t), 1),
             "median_rate": round(float(np.median([(h[-1] / h[0]) ** (1.0 / max(len(h) - 1, 1))
                                                   for h in hist])), 4),
             "sweep_cfg_rows": [b.sweep_config(l)[1] for l in range(3)]}
        if groups > 1:
            out[tag] = r
            del b, sts
            continue
        # kernel timing of the batched cycle: a few directly launched cycles
        b.profile(True)
        t0 = time.perf_counter()
        b.solve(10, 0.0, False)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        prof = b.profile_read()
        b.profile(False)
        r["cycle_ms_all_active"] = round(1e3 * t / 10, 3)
        r["kernel_ms_per_cycle"] = {k: round(v[0] / 10, 3) for k, v in prof.items()}
        if not fp32:
            ms, cnt = prof["sweep"]
            per_cycle = 3.0 * float(cells.sum()) * (1 + 0.25 + 0.0625) * SWEEP_BYTES_PER_CELL
            ach = per_cycle * 10 / (ms * 1e-3) / 1e9
            out["roofline_batched_sweep"] = {
                "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 5), "kernel": "k_sgs4, one launch per stage and level over "
                "all 64 cases", "avg_launch_us": round(1e3 * ms / max(cnt, 1), 3), "launches": cnt}
        out[tag] = r
        del b, sts
    # the grouping changes when cases run, not what they compute
    out["groups_bitwise_equal_to_one_group"] = all(
        np.array_equal(finals[t][k], finals[t + "_one_group"][k]) for t in ("fp32_precond", "fp64")
        for k in range(len(cases)))
    # converged solutions of the two precisions, cases that reached the drop in both
    u64, u32 = finals["fp64"], finals["fp32_precond"]
    # at the 6-order stop the two runs differ by their remaining iteration
    # error, not by the preconditioner precision (that is compared on
    # converged solutions in the single-case section)
    both = [k for k in range(len(cases)) if status["fp64"][k] == 0 and status["fp32_precond"][k] == 0]
    diffs = [float((np.abs(u32[k] - u64[k]).max(axis=0) / np.abs(u64[k]).max(axis=0)).max()) for k in both]
    out["fp32_vs_fp64_rel_state_diff_at_6_orders"] = (
        {"max": max(diffs), "median": float(np.median(diffs)), "cases": len(both)} if both else None)
    # FP64 per-case loop: the iterates are bitwise those of the FP64 batch
    # (same kernels, same order), so its time to the drop is the per-case
    # cycle time times the batch's per-case cycle count
    log("fp64 per-case loop (%s)" % ("full" if full_loop else "%d cycles per case" % loop_cycles))
    t_loop = 0.0
    per_case_ms = []
    if full_loop:
        t0 = time.perf_counter()
        for (g, u0), c in zip(grids, cases):
            st = fas.State(g, batch_params(fas, c, False), u0)
            st.cycle(cap, 6.0)
        torch.cuda.synchronize()
        t_loop = time.perf_counter() - t0
        out["fp64_per_case_loop"] = {"seconds": round(t_loop, 3), "estimated": False,
                                     "measured": "full solve of every case"}
    else:
        for (g, u0), c in zip(grids, cases):
            st = fas.State(g, batch_params(fas, c, False), u0)
            st.cycle(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.cycle(loop_cycles)
            torch.cuda.synchronize()
            per_case_ms.append(1e3 * (time.perf_counter() - t0) / loop_cycles)
        ms = np.array(per_case_ms)
        t_loop = float((cycles["fp64"] * ms).sum() * 1e-3)
        out["fp64_per_case_loop"] = {
            "seconds": round(t_loop, 3), "estimated": True,
            "measured": "ESTIMATE: cycle time of every case over %d cycles after 2 warm-up cycles, times the "
                        "case's cycle count to the drop (its iterates are bitwise those of the FP64 "
                        "batch)" % loop_cycles,
            "cell_cycles_per_s": round(float((cells * cycles["fp64"]).sum() / t_loop), 1)}
    out["speedup_fp32_batch_vs_fp64_loop"] = round(t_loop / out["fp32_precond"]["seconds"], 2)
    out["speedup_fp64_batch_vs_fp64_loop"] = round(t_loop / out["fp64"]["seconds"], 2)
    out["speedup_groups_vs_one_group"] = {
        "fp32_precond": round(out["fp32_precond_one_group"]["seconds"] / out["fp32_precond"]["seconds"], 3),
        "fp64": round(out["fp64_one_group"]["seconds"] / out["fp64"]["seconds"], 3)}
    return out


def unsteady_section(fas, torch, inner_cap):
    """Pitching airfoil on the moving mesh: 512 x 128 C-grid (n_w = 64), RANS,
    M = 0.8, alpha(t) = sin(2 k t) degrees with k = 0.2 (t in chords per free
    stream speed), dt = 0.460960, 10 BDF steps (the first implicit Euler),
    inner FAS V-cycles to an 11-order drop or the cap, from a steady start."""
    import numpy as np
    import fas_inputs as fi
    ni, nj, nw, mach = 512, 128, 64, 0.8
    x, y = fi.cgrid(ni, nj, nw)
    # the printed convective blocks diverge on this grid (measured): the
    # thin-layer viscous block term and the sum-form pseudo step are used
    par = fas.Params(model=fas.FAS_RANS_BL, scheme=fas.FAS_AW3, mach=mach, alpha_deg=0.0, reynolds=1e7,
                     n_levels=3, cycle_gamma=1, nu1=1, eta=0.5, d_cut=0.5, cfl=100.0, cfl_ramp=1.0,
                     n_ramp=4, ramp_growth=1.5, kappa2c=0.125, viscous_blocks=1, dt_form=0)
    g = fas.Grid(fi.CGRID, x, y, nw, 3)
    st = fas.State(g, par, torch.from_numpy(fi.uniform_state(ni, nj, mach, 0.0)).cuda())
    log("unsteady: steady start")
    h0, _ = st.cycle(400, 6.0)
    omega_t = 2 * 0.2 * mach * np.sqrt(1.4)
    dt = 0.460960
    steps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_cycles = 0
    for n in range(10):
        t = (n + 1) * dt
        st.set_motion(np.sin(omega_t * t), omega_t * np.cos(omega_t * t))
        h, status = st.dual_time_step(dt, 0.0, inner_cap, 11.0)
        total_cycles += len(h) - 1
        steps.append({"inner_cycles": len(h) - 1, "orders": round(float(np.log10(h[0] / h.min())), 2),
                      "rate": round(float((h[-1] / h[0]) ** (1.0 / max(len(h) - 1, 1))), 4),
                      "cl": round(st.forces()[0], 6)})
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return {"workload": "pitching RANS 512x128 C-grid, moving mesh, 10 BDF2 steps, inner V-cycles to "
                        "11 orders or %d cycles" % inner_cap,
            "steady_start": {"cycles": len(h0) - 1, "orders": round(float(np.log10(h0[0] / h0.min())), 2)},
            "seconds": round(t, 3), "inner_cycles": total_cycles,
            "cell_iters_per_s": round(ni * nj * total_cycles / t, 1),
            "mean_inner_rate": round(float(np.mean([s_["rate"] for s_ in steps])), 4),
            "steps": steps}


def unsteady_adjoint_section(fas, torch, inner_cap, adj_cap, steps=10, checkpoint_every=2):
    """The checkpointed unsteady adjoint on the 512 x 128 C-grid (n_w = 64),
    RANS, M = 0.8, fixed mesh with the far-field angle alpha(t) = sin(2 k t)
    degrees (k = 0.2), dt = 0.460960: the time-averaged lift over 10 BDF
    steps from the steady start and its gradient with respect to M and every
    step's angle, every second state kept (the others recomputed)."""
    import numpy as np
    import fas_inputs as fi
    ni, nj, nw, mach = 512, 128, 64, 0.8
    x, y = fi.cgrid(ni, nj, nw)
    par = fas.Params(model=fas.FAS_RANS_BL, scheme=fas.FAS_AW3, mach=mach, alpha_deg=0.0, reynolds=1e7,
                     n_levels=3, cycle_gamma=1, nu1=1, eta=0.5, d_cut=0.5, cfl=100.0, cfl_ramp=1.0,
                     n_ramp=4, ramp_growth=1.5, kappa2c=0.125, viscous_blocks=1, dt_form=0)
    g = fas.Grid(fi.CGRID, x, y, nw, 3)
    st = fas.State(g, par, torch.from_numpy(fi.uniform_state(ni, nj, mach, 0.0)).cuda())
    log("unsteady adjoint: steady start")
    h0, _ = st.cycle(400, 6.0)
    omega_t = 2 * 0.2 * mach * np.sqrt(1.4)
    dt = 0.460960
    alphas = [float(np.sin(omega_t * n * dt)) for n in range(steps + 1)]
    log("unsteady adjoint: %d steps forward, adjoint backward" % steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, dm, da, its, orders, rec = st.unsteady_lift_gradient(dt, alphas, max_inner=inner_cap, inner_drop=11.0,
                                                            checkpoint_every=checkpoint_every,
                                                            adj_max_iter=adj_cap, adj_drop=8.0)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return {"workload": "RANS 512x128 C-grid, fixed mesh, far-field angle sin(2kt) deg, %d BDF steps "
                        "(inner V-cycles to 11 orders or %d), time-averaged lift; adjoint solves to 8 orders "
                        "or %d iterations, every %d-th state kept" % (steps, inner_cap, adj_cap, checkpoint_every),
            "steady_start_orders": round(float(np.log10(h0[0] / np.nanmin(h0))), 2),
            "seconds": round(t, 3), "recomputed_steps": int(rec),
            "adjoint_iterations_per_step": [int(v) for v in its],
            "adjoint_orders_per_step": [round(float(v), 2) for v in orders],
            # the gradient means something only where the adjoint solves reached their drop
            "converged": bool((orders >= 8.0).all()),
            "J_mean_cl": J, "dJ_dmach": dm if (orders >= 8.0).all() else None,
            "dJ_dalpha_deg": [float(v) for v in da] if (orders >= 8.0).all() else None}


def unsteady_adjoint_c2_section(fas, torch, steps=10, checkpoint_every=2, adj_cap=2000):
    """The checkpointed unsteady adjoint on the 256 x 128 RANS workload, whose
    steady solve converges: the steady start to 11 orders, then 10 BDF steps
    with the far-field angle alpha_0 + sin(2 k t) degrees (k = 0.2, dt =
    0.460960, inner V-cycles to 11 orders or 300), the time-averaged lift and
    its gradient with respect to M and every step's angle; every adjoint
    solve to 8 orders or the cap, every second state kept.  The gradient is
    reported only if every adjoint solve reached its drop."""
    import numpy as np
    case, p = workload_params(fas, False)
    x, y = case.grid()
    g = fas.Grid(case.topology, x, y, case.n_wake, p.n_levels)
    st = fas.State(g, p, torch.from_numpy(case.initial_state(x, y)).cuda())
    log("unsteady adjoint 256x128: steady start to 11 orders")
    h0, s0 = st.cycle(3000, 11.0)
    omega_t = 2 * 0.2 * p.mach * np.sqrt(1.4)
    dt = 0.460960
    alphas = [p.alpha_deg + float(np.sin(omega_t * n * dt)) for n in range(steps + 1)]
    log("unsteady adjoint 256x128: %d steps forward, adjoint backward" % steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, dm, da, its, orders, rec = st.unsteady_lift_gradient(dt, alphas, max_inner=300, inner_drop=11.0,
                                                            checkpoint_every=checkpoint_every,
                                                            adj_max_iter=adj_cap, adj_drop=8.0)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ok = bool((orders >= 8.0).all())
    return {"workload": "RANS 256x128 C-grid (the throughput case), fixed mesh, far-field angle alpha0 + "
                        "sin(2kt) deg, %d BDF steps (inner V-cycles to 11 orders or 300), time-averaged lift; "
                        "adjoint solves to 8 orders or %d iterations, every %d-th state kept"
                        % (steps, adj_cap, checkpoint_every),
            "steady_start": {"cycles": len(h0) - 1, "status": int(s0),
                             "orders": round(float(np.log10(h0[0] / np.nanmin(h0))), 2)},
            "seconds": round(t, 3), "recomputed_steps": int(rec),
            "adjoint_iterations_per_step": [int(v) for v in its],
            "adjoint_orders_per_step": [round(float(v), 2) for v in orders],
            "converged": ok, "J_mean_cl": J, "dJ_dmach": dm if ok else None,
            "dJ_dalpha_deg": [float(v) for v in da] if ok else None}


def adjoint_section(fas, torch, primal_cap, adj_cap):
    """Discrete adjoint of the lift on the 1024 x 256 C-grid (n_w = 128),
    RANS, M = 0.8, alpha ~ U[0, 2] deg (seed 5), FP64 residual with the FP32
    preconditioner: the primal FAS cycles to an 8-order drop (or the cap),
    then one gradient of C_L with respect to M, alpha and every node (x, y)
    (the adjoint solve, GMRES right-preconditioned by the transposed
    smoother, to 8 orders or the iteration cap, then the node products), and
    the transposed residual product (fas_vjp) timed on its own over 20 calls
    on a seeded adjoint vector."""
    import numpy as np
    import fas_inputs as fi
    case = fi.steady_cgrid_case(1024, 256, 128, seed=5)
    x, y = case.grid()
    # the printed convective blocks diverge on this grid (measured): the
    # thin-layer viscous block term and the sum-form pseudo step are used
    par = fas.Params(model=fas.FAS_RANS_BL, scheme=fas.FAS_AW3, mach=case.mach, alpha_deg=case.alpha_deg,
                     reynolds=case.reynolds, n_levels=3, cycle_gamma=1, nu1=1, eta=0.5, d_cut=0.5, cfl=100.0,
                     cfl_ramp=1.0, n_ramp=4, ramp_growth=1.5, kappa2c=0.125, precond_fp32=1, viscous_blocks=1,
                     dt_form=0)
    g = fas.Grid(case.topology, x, y, case.n_wake, 3)
    st = fas.State(g, par, torch.from_numpy(case.initial_state(x, y)).cuda())
    torch.cuda.synchronize()
    log("adjoint: primal to 8 orders (1024x256)")
    t0 = time.perf_counter()
    hp, sp = st.cycle(primal_cap, 8.0)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    log("adjoint: lift gradient (M, alpha, every node)")
    t0 = time.perf_counter()
    cl, gp, dx, dy, ha, sa = st.lift_gradient_nodes(adj_cap, 8.0)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    gen = torch.Generator(device="cuda")
    gen.manual_seed(6)
    lam = torch.randn(st.shape(), dtype=torch.float64, device="cuda", generator=gen)
    st.vjp(lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        st.vjp(lam)
    torch.cuda.synchronize()
    tv = (time.perf_counter() - t0) / 20
    cells = case.ni * case.nj
    return {"workload": "steady RANS 1024x256 C-grid (n_w 128), M=0.8, alpha=%.4f deg, FP32 preconditioner; "
                        "dC_L/d(M, alpha, every node x and y)" % case.alpha_deg,
            "primal": {"seconds": round(tp, 3), "cycles": len(hp) - 1, "status": int(sp),
                       "orders": round(float(np.log10(hp[0] / np.nanmin(hp))), 2)},
            # the gradient's values mean nothing until the adjoint solve has
            # converged, so only its cost and progress are reported
            "gradient": {"seconds": round(tg, 3), "adjoint_iterations": len(ha) - 1, "status": int(sa),
                         "converged": bool(sa == 0),
                         "orders": round(float(np.log10(ha[0] / np.nanmin(ha))), 2) if len(ha) > 1 else None,
                         "ms_per_adjoint_iteration": round(1e3 * tg / max(len(ha) - 1, 1), 3),
                         "cl": round(cl, 6), "node_gradient_entries": int(dx.numel() + dy.numel())},
            "vjp": {"ms_per_call": round(1e3 * tv, 4), "cells": cells,
                    "cell_products_per_s": round(cells / tv, 1)}}


def adjoint_c2_section(fas, torch):
    """A converged discrete adjoint on the 256 x 128 RANS workload (the
    throughput case): the primal to 11 orders, the adjoint GMRES to 10
    orders, and its lift gradient checked against central differences of
    the frozen-turbulence primal (freeze_mut: the converged state's eddy
    viscosity kept, the model the adjoint differentiates), each perturbed
    solve started from the converged state and run to ten times its final
    residual norm.  C_L(M) is strongly curved at this transonic condition,
    so the Mach check extrapolates two step sizes (Richardson, O(h^2))."""
    import dataclasses
    import numpy as np
    case, p = workload_params(fas, False)
    x, y = case.grid()
    g = fas.Grid(case.topology, x, y, case.n_wake, p.n_levels)
    st = fas.State(g, p, torch.from_numpy(case.initial_state(x, y)).cuda())
    log("adjoint 256x128: primal to 11 orders")
    t0 = time.perf_counter()
    hp, sp = st.cycle(3000, 11.0)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    log("adjoint 256x128: lift gradient")
    t0 = time.perf_counter()
    cl0, grad, ha, sa = st.lift_gradient(3000, 10.0)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    u0 = st.get_state().clone()
    p0 = st.params
    h_end = st.cycle(0)[0][0]
    alpha, mach = p0.alpha_deg, p0.mach

    def cl(a, m):
        st.set_state(u0)
        st.set_params(dataclasses.replace(p0, alpha_deg=a, mach=m, freeze_mut=1))
        h0 = st.cycle(0)[0][0]
        h, s = st.cycle(6000, float(np.log10(h0 / (10.0 * h_end))))
        return st.forces()[0], int(s)

    log("adjoint 256x128: frozen-turbulence central differences")
    runs = {}
    for key, (a, m) in {"a+": (alpha + 2e-2, mach), "a-": (alpha - 2e-2, mach), "m1+": (alpha, mach + 1e-3),
                        "m1-": (alpha, mach - 1e-3), "m2+": (alpha, mach + 2e-3),
                        "m2-": (alpha, mach - 2e-3)}.items():
        runs[key] = cl(a, m)
    fd_a = (runs["a+"][0] - runs["a-"][0]) / 4e-2
    fd_m1 = (runs["m1+"][0] - runs["m1-"][0]) / 2e-3
    fd_m2 = (runs["m2+"][0] - runs["m2-"][0]) / 4e-3
    fd_m = (4.0 * fd_m1 - fd_m2) / 3.0
    return {"workload": "steady RANS 256x128 C-grid (the throughput case), M=%.1f, alpha=%.4f deg; "
                        "dC_L/d(alpha, M) by the discrete adjoint" % (mach, alpha),
            "primal": {"cycles": len(hp) - 1, "status": int(sp), "seconds": round(tp, 3),
                       "orders": round(float(np.log10(hp[0] / hp.min())), 2)},
            "adjoint": {"iterations": len(ha) - 1, "status": int(sa), "seconds": round(tg, 3),
                        "orders": round(float(np.log10(ha[0] / ha.min())), 2)},
            "cl": cl0, "dcl_dalpha_deg": float(grad[0]), "dcl_dmach": float(grad[1]),
            "frozen_turbulence_fd": {
                "dcl_dalpha_deg": fd_a, "alpha_step_deg": 2e-2,
                "rel_gap_alpha": abs(fd_a - grad[0]) / abs(fd_a),
                "dcl_dmach_steps_1e-3_2e-3": [fd_m1, fd_m2], "dcl_dmach_extrapolated": fd_m,
                "rel_gap_mach_extrapolated": abs(fd_m - grad[1]) / abs(fd_m),
                "solves_converged": all(v[1] == 0 for v in runs.values())}}


def _oracle_cycles(seconds_target):
    """The oracle (numpy + C sweep, one thread) on the first V-cycles of the
    workload: (cycles, seconds, fine cells)."""
    from threadpoolctl import threadpool_limits
    import fas_inputs as fi
    from oracle import fas as ofas
    case = fi.steady_cgrid_case()
    x, y = case.grid()
    u0 = case.initial_state(x, y)
    op = ofas.Params(model=1, scheme=0, mach=case.mach, alpha_deg=case.alpha_deg,
                     reynolds=case.reynolds, n_levels=3, cycle_gamma=1, nu1=1, eta=0.5, d_cut=0.5,
                     cfl=100.0, cfl_ramp=1.0, n_ramp=4, ramp_growth=1.5, kappa2c=0.125,
                     viscous_blocks=0, dt_form=1)
    with threadpool_limits(limits=1):
        S = ofas.Solver(x, y, case.topology, case.n_wake, op, u0)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < seconds_target and n < 200:
            S.cycle(0)
            S.n_cycles += 1
            n += 1
        t = time.perf_counter() - t0
    return n, t, case.ni * case.nj


def _oracle_worker(args):
    return _oracle_cycles(*args)


def cpu_baseline(seconds_target=12.0):
    """The oracle on the host's cores: one single-threaded oracle process per
    core (at most 16, the GPU machine's CPU share), each running the first
    V-cycles of the same workload for a fixed time; the value is their
    summed fine-cell cycles per second.  Runs before the GPU is touched (the
    workers are forked)."""
    import multiprocessing as mp
    cores = max(1, min(os.cpu_count() or 1, 16))
    os.environ["OMP_NUM_THREADS"] = "1"
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(seconds_target,)] * cores)
    one = res[0][0] * res[0][2] / res[0][1]
    total = sum(n * c / t for n, t, c in res)
    return {"value": round(total, 1), "unit": "fine-cell cycles/s", "cores": cores, "kind": "oracle",
            "one_core_value": round(one, 1),
            "sample": "%d independent single-threaded oracle processes, each running the first %d-%d FAS "
                      "V-cycles of the 256x128 RANS C-grid workload for about %.0f s (numpy + C sweep)"
                      % (cores, min(r[0] for r in res), max(r[0] for r in res), seconds_target)}


def kernels_only(fas, torch, which, cycles):
    """A few cycles of one workload and nothing else, for profiler runs
    (every dispatch is traced or counted): 'c2' / 'c2-fp32' is the 256 x 128
    RANS throughput case, 'batch' / 'batch-fp32' the 64-case batch with the
    default sweep configurations (no autotuning).  Cycles are launched
    directly, not from a captured graph."""
    if which.startswith("c2"):
        case, p = workload_params(fas, which.endswith("fp32"))
        x, y = case.grid()
        g = fas.Grid(case.topology, x, y, case.n_wake, p.n_levels)
        st = fas.State(g, p, torch.from_numpy(case.initial_state(x, y)).cuda())
        st.cycle(1)
        torch.cuda.synchronize()
        log("%s: %d cycles" % (which, cycles))
        st.profile(True)                 # per-launch events: keeps the cycles out of the graph
        st.cycle(cycles)
        st.profile(False)
    else:
        import fas_inputs as fi
        fp32 = which.endswith("fp32")
        cases = fi.batch_cases(64, seed=4)
        sts = []
        for c in cases:
            x, y = c.grid()
            sts.append(fas.State(fas.Grid(c.topology, x, y, c.n_wake, 3), batch_params(fas, c, fp32),
                                 torch.from_numpy(c.initial_state(x, y)).cuda()))
        b = fas.Batch(sts, autotune=False)
        b.solve(1, 0.0, False)
        torch.cuda.synchronize()
        log("%s: %d cycles" % (which, cycles))
        b.solve(cycles, 0.0, False)
    torch.cuda.synchronize()
    print(json.dumps({"kernels_only": which, "cycles": cycles}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--drop-cap", type=int, default=400)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-drop", action="store_true", help="skip the time-to-drop runs")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-case batched section")
    ap.add_argument("--batch-cap", type=int, default=1000)
    ap.add_argument("--loop-cycles", type=int, default=20)
    ap.add_argument("--full-loop", action="store_true",
                    help="solve every case of the FP64 per-case loop to the drop (minutes)")
    ap.add_argument("--no-unsteady", action="store_true", help="skip the pitching-airfoil section")
    ap.add_argument("--inner-cap", type=int, default=300)
    ap.add_argument("--unsteady-adjoint-cap", type=int, default=100,
                    help="adjoint iterations per step of the 512x128 unsteady adjoint")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB buffer 5 times (HBM counter calibration)")
    ap.add_argument("--no-dfa", action="store_true", help="skip the Fourier analysis section")
    ap.add_argument("--no-studies", action="store_true", help="skip the smoother comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 1024x256 adjoint section")
    ap.add_argument("--adjoint-only", action="store_true", help="run only the two adjoint sections")
    ap.add_argument("--primal-cap", type=int, default=1000)
    ap.add_argument("--adjoint-cap", type=int, default=200)
    ap.add_argument("--dfa-only", action="store_true", help="run only the Fourier analysis section")
    ap.add_argument("--kernels-only", choices=("c2", "c2-fp32", "batch", "batch-fp32"),
                    help="run only a few cycles of one workload (for rocprofv3 counter runs)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "CALF_DIR", "CALW_DIR"),
                    help="summarise four rocprofv3 --pmc output folders into the sweep's traffic record")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not (args.no_cpu or args.calibrate_copy or args.dfa_only or args.adjoint_only or args.kernels_only):
        log("cpu baseline (oracle, every host core, before the GPU is used)")
        cpu = cpu_baseline()
    import numpy as np
    import torch
    if args.calibrate_copy:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes_read": a.numel() * 8, "copies": 5}))
        return
    from paper_1710_04875_amd import fas
    fas.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.dfa_only:
        print(json.dumps({"dfa": dfa_section(fas, torch)}), flush=True)
        return
    if args.kernels_only:
        kernels_only(fas, torch, args.kernels_only, args.steps)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint_256x128_converged": adjoint_c2_section(fas, torch),
                          "adjoint_1024x256": adjoint_section(fas, torch, args.primal_cap, args.adjoint_cap)}),
              flush=True)
        return
    run_gpu.no_drop = args.no_drop
    log("fp64 preconditioner run")
    r64 = run_gpu(fas, torch, args.steps, args.warmup, False, args.drop_cap)
    case, p = r64["case"], r64["params"]
    roof = sweep_roofline(r64, case, p.n_levels)
    roof["traffic"] = load_traffic("k_sgs_c2_fp64")
    res_ms, res_n = r64["prof"]["residual"]
    line = {
        "metric": "AW3+SGS cell-iters/s & time to 6-order drop; FP32-precond vs FP64",
        "value": round(r64["value"], 1),
        "unit": "fine-cell cycles/s",
        "n_gpus": 1,
        "steps": r64["steps_done"],
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "steady RANS (Baldwin-Lomax) 256x128 C-grid, NACA 4-digit 10%% section, "
                               "M=0.8, alpha=%.4f deg, Re=1e7; FAS V-cycle 3 levels; AW3+SGS d=0.5 "
                               "eta=0.5 c*=100" % case.alpha_deg,
                   "fine_cells": case.ni * case.nj, "levels": p.n_levels, "step": "one FAS cycle"},
        "time_to_6_orders_fp64": r64["drop"],
        "kernel_ms_per_step_fp64": {k: round(v[0] / max(r64["prof_cycles"], 1), 4)
                                    for k, v in r64["prof"].items()},
        "residual_kernel": {"avg_launch_us": round(1e3 * res_ms / max(res_n, 1), 3),
                            "launches": res_n},
        "roofline": roof,
        "paper_context": {"steady_rate": 0.85, "unsteady_rate": 0.77,
                          "hardware": "Intel i7-3770 one core (uflo103, NACA 64A010 512x64)"},
    }
    log("block forms and cycle types (time to 6 orders)")
    line["block_forms_6_orders"] = block_forms_section(fas, torch, args.drop_cap)
    log("64x64 Euler box, single grid")
    line["box_64x64_single_grid"] = box_section(fas, torch)
    if not args.no_studies:
        log("smoother comparison (AW3, AW5J, AW51, AW52, pARK3J over c*)")
        from paper_1710_04875_amd import studies
        line["smoothers_256x128"] = studies.smoother_comparison()
    if not args.no_fp32:
        log("fp32 preconditioner run")
        r32 = run_gpu(fas, torch, args.steps, args.warmup, True, args.drop_cap)
        u64, u32 = r64["final_state"], r32["final_state"]
        diff = float((np.abs(u32 - u64).max(axis=0) / np.abs(u64).max(axis=0)).max())
        diff_deep = None
        if r64["deep"] and r32["deep"]:
            d64, d32 = r64["deep_state"], r32["deep_state"]
            diff_deep = float((np.abs(d32 - d64).max(axis=0) / np.abs(d64).max(axis=0)).max())
        line["fp32_precond"] = {
            "value": round(r32["value"], 1), "ms_per_step": round(r32["ms_per_step"], 4),
            "speedup_vs_fp64": round(r32["value"] / r64["value"], 3),
            "time_to_6_orders": r32["drop"],
            "max_rel_state_diff_vs_fp64_after_drop_run": diff,
            "max_rel_state_diff_vs_fp64_converged": diff_deep,
            "converged_orders": ({"fp64": r64["deep"]["orders"], "fp32": r32["deep"]["orders"]}
                                 if diff_deep is not None else None),
            "kernel_ms_per_step": {k: round(v[0] / max(r32["prof_cycles"], 1), 4)
                                   for k, v in r32["prof"].items()},
        }
    if not args.no_batch:
        line["batch_64_cases"] = batch_section(fas, torch, args.batch_cap, args.loop_cycles,
                                               args.full_loop)
    if not args.no_unsteady:
        line["unsteady_pitching"] = unsteady_section(fas, torch, args.inner_cap)
        line["unsteady_adjoint_512x128"] = unsteady_adjoint_section(fas, torch, 100, args.unsteady_adjoint_cap)
        line["unsteady_adjoint_256x128_converged"] = unsteady_adjoint_c2_section(fas, torch)
    if not args.no_dfa:
        log("discrete Fourier analysis")
        line["dfa"] = dfa_section(fas, torch)
    if not args.no_adjoint:
        line["adjoint_256x128_converged"] = adjoint_c2_section(fas, torch)
        line["adjoint_1024x256"] = adjoint_section(fas, torch, args.primal_cap, args.adjoint_cap)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
