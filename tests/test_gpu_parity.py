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
    cfl = 1.0 if scheme == 5 else 50.0
    g, st, S = make_pair(inp, scheme=scheme, cfl=cfl, cfl_ramp=cfl)
    st.smooth(0, 1)
    S.smooth(0)
    assert state_err(_np(st.get_state()), S.u(0)) < TOL_STATE
    levels = 2 if kind == "box_small" else 3
    g, st, S = make_pair(inp, scheme=scheme, n_levels=levels, cfl=cfl, cfl_ramp=cfl)
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
