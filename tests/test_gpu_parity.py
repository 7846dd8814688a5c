"""HIP library vs the FP64 oracle, element by element (needs a GPU)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import TOL_STATE, case_inputs, make_pair, res_err, state_err

pytestmark = pytest.mark.gpu

KINDS = ["box", "cgrid_small_euler", "cgrid_small_rans", "cgrid_c2_rans"]


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# box_small (ni > nj) and box_tall (ni < nj) take the two arrangements of the
# hyperplane-ordered cell numbering the cell kernels launch over
@pytest.mark.parametrize("kind", KINDS + ["box_small", "box_tall"])
def test_residual_parity(kind):
    inp = case_inputs(kind)
    g, st, S = make_pair(inp)
    Fg = _np(st.residual(0))
    Fo = S.residual(0)
    assert res_err(Fg, Fo) < 1e-12


@pytest.mark.parametrize("kind", ["box_small", "box_tall", "cgrid_small_euler", "cgrid_small_rans",
                                  "cgrid_c2_rans"])
def test_sgs_apply_parity(kind):
    inp = case_inputs(kind)
    g, st, S = make_pair(inp, cfl=1e4, cfl_ramp=1e4)
    nj, ni = inp["u0"].shape[1:]
    r = np.random.default_rng(5).standard_normal((4, nj, ni))
    xg = _np(st.sgs_apply(torch.from_numpy(r).cuda()))
    _, dts, mutp, B = S.prepare(0, cfl=1e4)
    xo = B.apply(r)
    assert res_err(xg, xo, floor=1e-9) < 1e-11


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("scheme", [0, 1])
def test_one_smoother_iteration(kind, scheme):
    inp = case_inputs(kind)
    cfl = 1e4 if scheme == 0 else 1.0
    g, st, S = make_pair(inp, scheme=scheme, cfl=cfl, cfl_ramp=cfl)
    st.smooth(0, 1)
    S.smooth(0)
    assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE


@pytest.mark.parametrize("kind", ["cgrid_small_rans", "cgrid_c2_rans"])
@pytest.mark.parametrize("vblk,dt_form", [(0, 1), (1, 1), (0, 0)])
def test_one_iteration_both_block_forms(kind, vblk, dt_form):
    """One AW3 iteration on RANS grids with the printed convective blocks
    (viscous_blocks 0) and with the thin-layer viscous term (1), and with
    both pseudo-time-step readings."""
    inp = case_inputs(kind)
    g, st, S = make_pair(inp, cfl=1e4, cfl_ramp=1e4, viscous_blocks=vblk, dt_form=dt_form)
    st.smooth(0, 1)
    S.smooth(0)
    assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE


@pytest.mark.parametrize("vblk", [0, 1])
def test_c2_size_v_cycle_both_block_forms(vblk):
    """One 3-level V-cycle on the 256 x 128 RANS C-grid (the benchmark's
    grid size and banded sweeps on every level) in both block forms; every
    level is compared."""
    inp = case_inputs("cgrid_c2_rans")
    # c* = 1, the benchmark's start-up value (the perturbed parity state
    # diverges at large c* in both paths)
    g, st, S = make_pair(inp, n_levels=3, cycle_gamma=1, cfl=1.0, cfl_ramp=1.0, viscous_blocks=vblk)
    hist, status = st.cycle(1)
    ho = S.run_cycles(1)
    assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE
    for l in range(1, 3):
        ug, sg = st.get_level(l)
        assert state_err(_np(ug), S.u(l)) < TOL_STATE
    assert abs(hist[1] - ho[1]) <= 1e-10 * ho[1]


def test_c5_size_v_cycle():
    """One 3-level V-cycle on the 1024 x 256 RANS C-grid of the adjoint
    workload (262,144 fine cells: the tiled residual, the one-lane block
    kernel and the banded sweeps of a 256-row grid), with the thin-layer
    viscous blocks and the sum-form pseudo step that workload runs; every
    level is compared."""
    inp = case_inputs("cgrid_c5_rans")
    g, st, S = make_pair(inp, n_levels=3, cycle_gamma=1, cfl=1.0, cfl_ramp=1.0, viscous_blocks=1, dt_form=0)
    hist, status = st.cycle(1)
    ho = S.run_cycles(1)
    assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE
    for l in range(1, 3):
        ug, sg = st.get_level(l)
        assert state_err(_np(ug), S.u(l)) < TOL_STATE
    assert abs(hist[0] - ho[0]) <= 1e-12 * ho[0]
    assert abs(hist[1] - ho[1]) <= 1e-10 * ho[1]


@pytest.mark.parametrize("kind,levels,gamma", [("box_small", 2, 1), ("cgrid_small_rans", 3, 1),
                                               ("cgrid_small_euler", 3, 2)])
def test_one_fas_cycle(kind, levels, gamma):
    inp = case_inputs(kind)
    g, st, S = make_pair(inp, n_levels=levels, cycle_gamma=gamma, cfl=20.0, cfl_ramp=20.0)
    hist, status = st.cycle(1)
    ho = S.run_cycles(1)
    assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE
    for l in range(1, levels):
        ug, sg = st.get_level(l)
        assert state_err(_np(ug), S.u(l)) < TOL_STATE
    assert abs(hist[0] - ho[0]) <= 1e-12 * ho[0]
    assert abs(hist[1] - ho[1]) <= 1e-10 * ho[1]


def test_convergence_rate_parity():
    """Twenty V-cycles on the RANS C-grid: per-cycle residual histories agree
    and the average rate agrees within 0.01."""
    inp = case_inputs("cgrid_small_rans")
    par = dict(n_levels=3, cfl=1e4, cfl_ramp=1.0, n_ramp=4, ramp_growth=1.5)
    g, st, S = make_pair(inp, **par)
    n = 20
    hist, status = st.cycle(n)
    ho = S.run_cycles(n)
    rg = (hist[-1] / hist[0]) ** (1.0 / n)
    ro = (ho[-1] / ho[0]) ** (1.0 / n)
    assert abs(rg - ro) < 0.01
    assert np.allclose(hist, ho, rtol=1e-6)


def test_dual_time_step_parity():
    inp = case_inputs("cgrid_small_rans")
    g, st, S = make_pair(inp, n_levels=2, cfl=20.0, cfl_ramp=20.0)
    dt = 0.46096
    for step, alpha in enumerate([1.3, 1.35]):
        hist, status = st.dual_time_step(dt, alpha, 2, 0.0)
        S.begin_time_step(dt, alpha)
        S.run_cycles(2)
        assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE, step


@pytest.mark.parametrize("kind", ["box_small", "cgrid_small_rans"])
@pytest.mark.parametrize("scheme", [2, 3, 4, 5])
def test_five_stage_smoothers(kind, scheme):
    """AW5J, AW51, AW52 and pARK51 (the five-stage rows of the coefficient
    table) run on the same kernels: one iteration and one V-cycle."""
    inp = case_inputs(kind)
    cfl = 0.5 if scheme == 5 else 50.0
    g, st, S = make_pair(inp, scheme=scheme, cfl=cfl, cfl_ramp=cfl)
    st.smooth(0, 1)
    S.smooth(0)
    assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE
    levels = 2 if kind == "box_small" else 3
    # the V-cycle on the RANS C-grid with the viscous block term (with the
    # convective blocks alone these c* diverge on its coarse levels)
    g, st, S = make_pair(inp, scheme=scheme, n_levels=levels, cfl=cfl, cfl_ramp=cfl,
                         viscous_blocks=1 if kind.endswith("rans") else 0)
    st.cycle(1)
    S.run_cycles(1)
    assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE


@pytest.mark.parametrize("kind", ["cgrid_small_euler", "cgrid_small_rans"])
def test_pitching_moving_mesh_parity(kind):
    """Rigid-body pitching on the moving mesh: two BDF time steps with the
    mesh turned and spinning, two inner V-cycles each."""
    inp = case_inputs(kind)
    g, st, S = make_pair(inp, n_levels=2, cfl=20.0, cfl_ramp=20.0)
    dt, amp, om = 0.46096, 1.01, 0.4
    for step in range(2):
        t = (step + 1) * dt
        da, rate = amp * np.sin(om * t), amp * om * np.cos(om * t)
        st.set_motion(da, rate)
        hist, status = st.dual_time_step(dt, inp["alpha"], 2, 0.0)
        S.begin_time_step(dt, inp["alpha"])
        S.set_motion(da, rate)
        S.run_cycles(2)
        assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE, step


@pytest.mark.parametrize("kind", ["cgrid_small_rans", "cgrid_c2_rans", "cgrid_c5_rans", "box"])
def test_fp32_preconditioner_iteration_against_oracle(kind):
    """One AW3 iteration with the FP32 preconditioner (blocks, D^-1, both
    sweeps and x in FP32; residual and update in FP64) against the FP64
    oracle.  The FP32 path changes only x, the increment of the iteration,
    so the difference is measured against the increment's size per
    component; the bound is FP32_INCREMENT_TOL (derivation in the design
    notes: FP32 rounding, u32 = 6e-8, of the blocks, of g and of every
    sweep product, carried along the sweep's dependency chain; measured
    0.9e-6 to 1.8e-6 on these grids)."""
    inp = case_inputs(kind)
    g, st, S = make_pair(inp, cfl=100.0, cfl_ramp=100.0, precond_fp32=1)
    st.smooth(0, 1)
    S.smooth(0)
    ug = _np(st.get_state())
    uo = S.u(0)
    inc = np.abs(uo - inp["u0"]).max(axis=(1, 2))
    err = float((np.abs(ug - uo).max(axis=(1, 2)) / inc).max())
    print("fp32 increment error %s: %.3e" % (kind, err))
    assert err < FP32_INCREMENT_TOL


FP32_INCREMENT_TOL = 2e-5


def test_fp32_and_fp64_preconditioners_converge_to_the_same_solution():
    """The 256 x 128 RANS C-grid solved to 11 orders with the FP32 and with
    the FP64 preconditioner (W-cycles): the fixed point F(u) = 0 does not
    depend on the preconditioner's precision (within 1e-8 per cell)."""
    import fas_inputs as fi
    from paper_1710_04875_amd import fas
    case = fi.steady_cgrid_case()
    x, y = case.grid()
    u0 = torch.from_numpy(case.initial_state(x, y)).cuda()
    out = []
    for fp32 in (0, 1):
        g = fas.Grid(case.topology, x, y, case.n_wake, 3)
        p = fas.Params(model=fas.FAS_RANS_BL, mach=case.mach, alpha_deg=case.alpha_deg, reynolds=case.reynolds,
                       n_levels=3, cycle_gamma=2, cfl=100.0, cfl_ramp=1.0, n_ramp=4, ramp_growth=1.5,
                       precond_fp32=fp32)
        st = fas.State(g, p, u0)
        h, status = st.cycle(1500, 11.0)
        print("precision fp32=%d: %d cycles, %.2f orders" % (fp32, len(h) - 1, np.log10(h[0] / h[-1])))
        assert status == fas.FAS_OK
        out.append(_np(st.get_state()))
    assert state_err(out[1], out[0]) < 1e-8


def test_c3_size_pitching_steps():
    """The pitching workload's grid at full size (512 x 128 RANS C-grid,
    3 levels, viscous blocks and the sum-form pseudo step as that workload
    runs them): two BDF time steps on the turning, spinning mesh, one inner
    V-cycle each, against the oracle on every level."""
    inp = case_inputs("cgrid_c3_rans")
    g, st, S = make_pair(inp, n_levels=3, cycle_gamma=1, cfl=1.0, cfl_ramp=1.0, viscous_blocks=1, dt_form=0)
    dt, amp, om = 0.46096, 1.0, 0.4
    for step in range(2):
        t = (step + 1) * dt
        da, rate = amp * np.sin(om * t), amp * om * np.cos(om * t)
        st.set_motion(da, rate)
        st.dual_time_step(dt, inp["alpha"], 1, 0.0)
        S.begin_time_step(dt, inp["alpha"])
        S.set_motion(da, rate)
        S.run_cycles(1)
        assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE, step
    for l in range(1, 3):
        ug, sg = st.get_level(l)
        assert state_err(_np(ug), S.u(l)) < TOL_STATE


def test_c1_box_fifty_iterations():
    """The single-grid smoother workload as the benchmark runs it: the 64 x 64
    jittered Euler box from the bump-and-noise state, 50 AW3 iterations with
    the SGS preconditioner (d 0.5, eta 0.5, c* 20 for two iterations, then
    1e4); the state after all 50 and the residual history against the
    oracle."""
    inp = case_inputs("box")
    g, st, S = make_pair(inp, n_levels=1, eta=0.5, d_cut=0.5, cfl=1.0e4, cfl_ramp=20.0, n_ramp=2)
    hist, status = st.cycle(50)
    ho = S.run_cycles(50)
    assert len(hist) == len(ho) == 51
    assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE
    assert np.allclose(hist, ho, rtol=1e-10, atol=0.0)
