"""Shared helpers for the GPU parity tests: build the same case on the HIP
library and in the oracle from one set of seeded inputs."""
import numpy as np

import fas_inputs as fi

TOL_STATE = 1e-12       # max_k |du_k| / max_k |u_k| per cell
TOL_RES_FLOOR = 1e-10   # residual arrays: relative to max(|R_c|, floor * max|R|)


def case_inputs(kind):
    if kind == "box":
        x, y = fi.box_grid(64, 64)
        return dict(topo=fi.BOX, x=x, y=y, nw=0, u0=fi.box_initial_state(x, y), model=0,
                    alpha=0.0)
    if kind == "box_tall":         # nj > 256: the one-thread-per-row sweep
        x, y = fi.box_grid(16, 288, ratio=1.01)
        return dict(topo=fi.BOX, x=x, y=y, nw=0, u0=fi.box_initial_state(x, y), model=0,
                    alpha=0.0)
    if kind == "box_small":
        x, y = fi.box_grid(24, 20)
        return dict(topo=fi.BOX, x=x, y=y, nw=0, u0=fi.box_initial_state(x, y), model=0,
                    alpha=0.0)
    ni, nj, nw = {"cgrid_small": (64, 32, 8), "cgrid_mid": (128, 64, 16),
                  "cgrid_c2": (256, 128, 32), "cgrid_c3": (512, 128, 64),
                  "cgrid_c5": (1024, 256, 128)}[kind.rsplit("_", 1)[0] if kind.endswith(("_euler", "_rans")) else kind]
    x, y = fi.cgrid(ni, nj, nw)
    model = 0 if kind.endswith("_euler") else 1
    u0 = fi.perturbed_state(fi.uniform_state(ni, nj, 0.8, 1.3), 0.01, seed=11)
    return dict(topo=fi.CGRID, x=x, y=y, nw=nw, u0=u0, model=model, alpha=1.3)


def make_pair(inp, n_levels=1, **par):
    import torch
    from paper_1710_04875_amd import fas
    from oracle import fas as ofas
    kw = dict(model=inp["model"], mach=0.8, alpha_deg=inp["alpha"], n_levels=n_levels)
    kw.update(par)
    gp = fas.Params(**{k: v for k, v in kw.items() if k in fas.Params.__dataclass_fields__})
    op = ofas.Params(**{k: v for k, v in kw.items() if k in ofas.Params.__dataclass_fields__})
    g = fas.Grid(inp["topo"], inp["x"], inp["y"], inp["nw"], n_levels)
    st = fas.State(g, gp, torch.from_numpy(inp["u0"]).cuda())
    S = ofas.Solver(inp["x"], inp["y"], inp["topo"], inp["nw"], op, inp["u0"])
    return g, st, S


def state_err(ug, uo):
    return float((np.abs(ug - uo).max(axis=0) / np.abs(uo).max(axis=0)).max())


def res_err(Fg, Fo, floor=TOL_RES_FLOOR):
    cell = np.abs(Fo).max(axis=0)
    den = np.maximum(cell, floor * cell.max())
    return float((np.abs(Fg - Fo).max(axis=0) / den).max())
