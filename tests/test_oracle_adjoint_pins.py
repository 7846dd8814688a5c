"""Pins of the oracle's discrete adjoint against facts that do not come from
the adjoint code itself: central differences of the residual, the closure
of the airfoil surface, and the direct (forward) sensitivity (CPU only)."""
import numpy as np
import pytest

import fas_inputs as fi
from oracle import adjoint as adj
from oracle import fas


def _state(model, ni=32, nj=16, nw=4, mach=0.7, alpha=1.3, seed=11):
    x, y = fi.cgrid(ni, nj, nw)
    u = fi.perturbed_state(fi.uniform_state(ni, nj, mach, alpha), 0.01, seed=seed)
    S = fas.Solver(x, y, fi.CGRID, nw, fas.Params(model=model, mach=mach, alpha_deg=alpha), u)
    return S, u


@pytest.mark.parametrize("model", [0, 1])
def test_complex_step_product_matches_central_differences(model):
    S, u = _state(model)
    mutp = adj.frozen_mut(S, u)
    v = np.random.default_rng(0).standard_normal(u.shape)
    jv = adj.fine_residual(S, u + 1j * adj.H_CS * v, mutp).imag / adj.H_CS
    h = 1e-6
    fd = (adj.fine_residual(S, u + h * v, mutp) - adj.fine_residual(S, u - h * v, mutp)) / (2 * h)
    assert np.abs(jv - fd).max() <= 1e-8 * np.abs(jv).max()
    # the real part of the complex evaluation is the residual itself (up to
    # the rounding of complex division)
    F = adj.fine_residual(S, u + 1j * adj.H_CS * v, mutp).real
    F0 = S.residual(0)
    assert np.abs(F - F0).max() <= 1e-14 * np.abs(F0).max()


def test_dense_jacobian_columns_are_directional_derivatives():
    S, u = _state(1, ni=16, nj=8, nw=2)
    mutp = adj.frozen_mut(S, u)
    J = adj.dense_jacobian(S, u, mutp)
    v = np.random.default_rng(1).standard_normal(u.shape)
    jv = adj.fine_residual(S, u + 1j * adj.H_CS * v, mutp).imag / adj.H_CS
    assert np.abs(J @ v.reshape(-1) - jv.reshape(-1)).max() <= 1e-12 * np.abs(jv).max()


@pytest.mark.parametrize("model", [0, 1])
def test_parameter_derivatives_match_central_differences(model):
    S, u = _state(model)
    mutp = adj.frozen_mut(S, u)
    da, dm = adj.residual_param_partials(S, u, mutp)
    h = 1e-5
    fa = (adj.fine_residual(S, u, mutp, alpha_deg=1.3 + h)
          - adj.fine_residual(S, u, mutp, alpha_deg=1.3 - h)) / (2 * h)
    fm = (adj.fine_residual(S, u, mutp, mach=0.7 + h) - adj.fine_residual(S, u, mutp, mach=0.7 - h)) / (2 * h)
    assert np.abs(da - fa).max() <= 1e-6 * np.abs(da).max()
    assert np.abs(dm - fm).max() <= 1e-6 * np.abs(dm).max()


def test_uniform_pressure_exerts_no_force_on_the_closed_airfoil():
    x, y = fi.cgrid(64, 32, 8)
    for alpha in (0.0, 2.0):
        u = fi.uniform_state(64, 32, 0.7, alpha)
        S = fas.Solver(x, y, fi.CGRID, 8, fas.Params(model=0, mach=0.7, alpha_deg=alpha), u)
        cl, cd = adj.forces(S, u)
        assert abs(cl) < 1e-12 and abs(cd) < 1e-12


def test_lift_partials_match_central_differences():
    S, u = _state(0)
    g, cla, clm = adj.lift_partials(S, u)
    v = np.random.default_rng(2).standard_normal(u.shape)
    h = 1e-6
    fd = (adj.forces(S, u + h * v)[0] - adj.forces(S, u - h * v)[0]) / (2 * h)
    assert abs(np.sum(g * v) - fd) <= 1e-7 * abs(fd)
    fa = (adj.forces(S, u, alpha_deg=1.3 + 1e-5)[0] - adj.forces(S, u, alpha_deg=1.3 - 1e-5)[0]) / 2e-5
    assert abs(cla - fa) <= 1e-7 * abs(fa)


@pytest.mark.parametrize("model", [0, 1])
def test_adjoint_gradient_equals_direct_sensitivity(model):
    """dC_L/dq = dC_L/dq|_u + g . du/dq with J du/dq = -dF/dq (direct)
    equals the adjoint form dC_L/dq|_u + lam . dF/dq, J^T lam = -g."""
    S, u = _state(model, ni=16, nj=8, nw=2)
    mutp = adj.frozen_mut(S, u)
    J = adj.dense_jacobian(S, u, mutp)
    g, cla, clm = adj.lift_partials(S, u)
    da, dm = adj.residual_param_partials(S, u, mutp)
    (ga, gm), lam = adj.lift_gradient(S, u)
    dua = np.linalg.solve(J, -da.reshape(-1))
    dum = np.linalg.solve(J, -dm.reshape(-1))
    assert abs(ga - (cla + g.reshape(-1) @ dua)) <= 1e-8 * abs(ga)
    assert abs(gm - (clm + g.reshape(-1) @ dum)) <= 1e-8 * abs(gm)


def _spacing(x, y):
    """Smallest edge length at every node (scales test displacements, so
    that the displaced grids stay valid at wall spacings of 1e-6)."""
    sp = np.full(x.shape, np.inf)
    di = np.hypot(np.diff(x, axis=1), np.diff(y, axis=1))
    dj = np.hypot(np.diff(x, axis=0), np.diff(y, axis=0))
    sp[:, :-1] = np.minimum(sp[:, :-1], di)
    sp[:, 1:] = np.minimum(sp[:, 1:], di)
    sp[:-1, :] = np.minimum(sp[:-1, :], dj)
    sp[1:, :] = np.minimum(sp[1:, :], dj)
    return sp


@pytest.mark.parametrize("model", [0, 1])
def test_node_derivative_of_residual_matches_central_differences(model):
    S, u = _state(model)
    mutp = adj.frozen_mut(S, u)
    x, y = S.levels[0].x, S.levels[0].y
    sp = _spacing(x, y)
    rng = np.random.default_rng(4)
    vx, vy = rng.standard_normal(x.shape) * sp, rng.standard_normal(x.shape) * sp
    jv = adj.residual_node_jvp(S, u, mutp, vx, vy)
    h = 1e-5
    fd = (adj.residual_at_nodes(S, u, mutp, x + h * vx, y + h * vy)
          - adj.residual_at_nodes(S, u, mutp, x - h * vx, y - h * vy)) / (2 * h)
    assert np.abs(jv - fd).max() <= 2e-6 * np.abs(jv).max()
    # on the unperturbed nodes the residual is the solver's own
    F0 = adj.residual_at_nodes(S, u, mutp, x, y)
    assert np.array_equal(F0, adj.fine_residual(S, u, mutp))


@pytest.mark.parametrize("model", [0, 1])
def test_translating_the_grid_changes_neither_residual_nor_lift(model):
    """F and C_L depend on node differences only (the turbulence model's
    wall distance is frozen): a rigid translation has zero derivative."""
    S, u = _state(model)
    mutp = adj.frozen_mut(S, u)
    x = S.levels[0].x
    one, zero = np.ones(x.shape), np.zeros(x.shape)
    scale = np.abs(adj.residual_node_jvp(S, u, mutp, *(np.random.default_rng(5).standard_normal((2,) + x.shape)))).max()
    for v in ((one, zero), (zero, one)):
        assert np.abs(adj.residual_node_jvp(S, u, mutp, *v)).max() <= 1e-13 * scale
        assert abs(adj.lift_node_jvp(S, u, *v)) <= 1e-13


def test_node_derivative_of_lift_matches_central_differences():
    S, u = _state(0)
    x, y = S.levels[0].x, S.levels[0].y
    sp = _spacing(x, y)
    rng = np.random.default_rng(6)
    vx, vy = rng.standard_normal(x.shape) * sp, rng.standard_normal(x.shape) * sp
    h = 1e-5
    fd = (adj.forces(S, u, nodes=(x + h * vx, y + h * vy))[0]
          - adj.forces(S, u, nodes=(x - h * vx, y - h * vy))[0]) / (2 * h)
    # the derivative along this displacement is ~1e-6 while C_L ~ 0.1: the
    # central difference carries ~1e-16 * 0.1 / h of cancellation error
    assert abs(adj.lift_node_jvp(S, u, vx, vy) - fd) <= 1e-4 * abs(fd)


@pytest.mark.parametrize("model", [0, 1])
def test_adjoint_node_derivative_equals_direct_sensitivity(model):
    """dC_L/dX v = dC_L/dX|_u v + g . du with J du = -(dF/dX) v (direct)
    equals the adjoint form used for the node gradient."""
    S, u = _state(model, ni=16, nj=8, nw=2)
    mutp = adj.frozen_mut(S, u)
    x = S.levels[0].x
    rng = np.random.default_rng(7)
    vx, vy = rng.standard_normal((2,) + x.shape) * _spacing(x, S.levels[0].y)
    J = adj.dense_jacobian(S, u, mutp)
    g, _, _ = adj.lift_partials(S, u)
    du = np.linalg.solve(J, -adj.residual_node_jvp(S, u, mutp, vx, vy).reshape(-1))
    direct = adj.lift_node_jvp(S, u, vx, vy) + g.reshape(-1) @ du
    assert abs(adj.lift_node_derivative(S, u, vx, vy) - direct) <= 1e-8 * abs(direct)


@pytest.mark.parametrize("model,scheme", [(1, 0), (0, 1)])
def test_smoother_jacobian_matches_central_differences(model, scheme):
    """The complex-step Jacobian of one smoother iteration at frozen dt*,
    blocks and eddy viscosity against central differences of the same map
    (a perturbed C-grid state, away from the kinks of the switches)."""
    x, y = fi.cgrid(16, 8, 2)
    u = fi.perturbed_state(fi.uniform_state(16, 8, 0.7, 1.3), 0.01, seed=11)
    cfl = 1.0 if scheme == 1 else 50.0
    S = fas.Solver(x, y, fi.CGRID, 2, fas.Params(model=model, mach=0.7, alpha_deg=1.3, scheme=scheme,
                                                 cfl=cfl, cfl_ramp=cfl), u)
    J = adj.smoother_jacobian(S, u)
    frozen = S.prepare(0)
    v = np.random.default_rng(3).standard_normal(u.shape)
    h = 1e-7
    fd = (adj.smoother_map(S, u + h * v, frozen) - adj.smoother_map(S, u - h * v, frozen)) / (2 * h)
    assert np.abs(J @ v.reshape(-1) - fd.reshape(-1)).max() < 1e-7 * np.abs(fd).max()


def _unsteady_setup(mach, alpha0):
    """16 x 8 Euler C-grid: the steady start converged by 2-level V-cycles,
    the physical steps on one level (whose inner solves converge quickly)."""
    x, y = fi.cgrid(16, 8, 2)
    p2 = fas.Params(model=0, mach=mach, alpha_deg=alpha0, n_levels=2, cfl=10.0, cfl_ramp=5.0, n_ramp=1,
                    ramp_growth=1.5, dt_form=0)
    S = fas.Solver(x, y, fi.CGRID, 2, p2, fi.uniform_state(16, 8, mach, alpha0))
    S.run_cycles(3000, 13.0)
    p1 = fas.Params(**{**p2.__dict__, "n_levels": 1})
    return fas.Solver(x, y, fi.CGRID, 2, p1, S.u(0))


def test_unsteady_direct_gradient_matches_central_differences():
    """Dual time stepping (implicit Euler start, then BDF2; eq.
    "nonlin-eq"): the forward-sensitivity gradient of the time-averaged lift
    equals central differences of whole runs for the angle of the first
    step (the Mach number, which also moves the steady start, is checked by
    central differences on the GPU, where the runs are cheap)."""
    dt, mach, alphas = 0.1, 0.5, [1.0, 1.3, 1.6]

    def J_of(m, al, S=None):
        S = _unsteady_setup(m, al[0]) if S is None else S
        # the inner solves of this tiny grid settle into a limit cycle of
        # the sensor switches at about 3e-11 (7.5 orders below the step's
        # first norm): they stop at 7 orders
        st = adj.unsteady_states(S, dt, al, 1500, 7.0)
        return np.mean([adj.forces(S, u, mach=m, alpha_deg=a)[0] for u, a in zip(st[1:], al[1:])]), st

    S0 = _unsteady_setup(mach, alphas[0])
    u0 = S0.u(0)
    J, states = J_of(mach, alphas, S0)
    Jd, dm, da = adj.unsteady_direct_gradient(S0, states, dt, alphas)
    assert abs(Jd - J) < 1e-14
    ha = 1e-3
    x, y = fi.cgrid(16, 8, 2)

    def from_start(al):
        S = fas.Solver(x, y, fi.CGRID, 2, S0.par.__class__(**{**S0.par.__dict__, "alpha_deg": al[0]}), u0)
        return J_of(mach, al, S)[0]

    fd_a1 = (from_start([1.0, 1.3 + ha, 1.6]) - from_start([1.0, 1.3 - ha, 1.6])) / (2 * ha)
    # central differences of inner solves stopped at 7 orders: O(h^2) and
    # O(1e-11 / h) errors, both below 1e-4 of the derivative here
    assert abs(da[1] - fd_a1) <= 1e-4 * abs(fd_a1)
