"""Pins of the oracle's fluid-structure pieces: surface force (paper Sec. III),
the rigid-body ODEs (Sec. IV), the Grad wall boundary condition (Sec. III.A)
and whole-step symmetry / fixed-body properties."""

import math

import numpy as np
import pytest

import synth
from oracle import body as B
from oracle import lattice as L
from oracle import mesh as M
from oracle.boundary import wall_grad_bc
from oracle.forces import wall_force
from oracle.solver import OracleSolver


# ---- P14: surface force ------------------------------------------------------

def polygon_area(x, y):
    return 0.5 * abs(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


@pytest.mark.parametrize("theta", [0.0, 0.4, 2.0])
def test_force_of_linear_pressure_is_minus_gradient_times_area(theta):
    """A pressure field p = p0 + beta . x at rest gives F = -beta A_polygon
    exactly (discrete divergence theorem of the lumped normals); a uniform
    pressure gives F = M = 0; rotating the mesh and the gradient rotates F."""
    mesh = synth.ogrid_mesh(8, 64, 20.0, 0.5, 40.0)
    c, s = math.cos(theta), math.sin(theta)
    X = c * mesh.X - s * mesh.Y
    Y = s * mesh.X + c * mesh.Y
    grid = M.Grid(64, 8, 1)
    T0 = 0.3
    beta = np.array([c * 1e-3, s * 1e-3])
    for b, expect_zero in ((np.zeros(2), True), (beta, False)):
        p = 1.0 * T0 + b[0] * X + b[1] * Y
        rho = p / T0
        f, g = L.equilibrium_populations(rho, 0 * X, 0 * X, np.full_like(X, T0), 1.4)
        Fx, Fy, Mz = wall_force(grid, f, g, X, Y, 1.4, 0.02, 0.71, 0.5, (0.0, 0.0))
        if expect_zero:
            assert abs(Fx) < 1e-13 and abs(Fy) < 1e-13 and abs(Mz) < 1e-11
        else:
            A = polygon_area(X[0], Y[0])
            assert Fx == pytest.approx(-b[0] * A, rel=1e-10, abs=1e-14)
            assert Fy == pytest.approx(-b[1] * A, rel=1e-10, abs=1e-14)


def test_force_viscous_part_uses_nonequilibrium_stress():
    """A non-equilibrium shear stress P^(1)_xy = tau0 + beta x at uniform p
    gives the traction -(1 - omega/2) P^(1) . n, whose discrete divergence
    theorem on the lumped normals yields F = (0, -(1 - omega/2) beta A)."""
    mesh = synth.ogrid_mesh(4, 96, 20.0, 0.5, 30.0)
    X, Y = mesh.X, mesh.Y
    grid = M.Grid(96, 4, 1)
    T0 = 1 / 3
    f, g = L.equilibrium_populations(np.ones_like(X), 0 * X, 0 * X,
                                     np.full_like(X, T0), 1.4)
    tau0, beta = 2e-4, 1e-5
    tau = tau0 + beta * X
    for i in range(9):
        f[i] += tau * L.CX[i] * L.CY[i] / 4.0      # adds P_xy = tau, nothing else
    mu, Pr, dt = 0.02, 0.71, 0.5
    omega = 1 / (mu / (T0 * dt) + 0.5)             # mu = (1/omega - 1/2) p dt
    Fx, Fy, Mz = wall_force(grid, f, g, X, Y, 1.4, mu, Pr, dt, (0.0, 0.0))
    A = polygon_area(X[0], Y[0])
    assert abs(Fx) < 1e-14
    assert Fy == pytest.approx(-(1 - 0.5 * omega) * beta * A, rel=1e-10)


# ---- P15: rigid-body ODEs ----------------------------------------------------

def test_heave_free_vibration_and_rk4_order():
    body = synth.BodyParams(dof=1, m=2.0, k_h=3.0, h0=0.7)
    w = math.sqrt(3.0 / 2.0)
    errs = []
    for dt in (0.04, 0.02):
        s = B.initial_state(body)
        n = int(round(10.0 / dt))
        worst = 0.0
        for k in range(1, n + 1):
            s = B.rk4_step(body, s, 0.0, 0.0, dt)
            worst = max(worst, abs(s[0] - 0.7 * math.cos(w * k * dt)))
        errs.append(worst)
    order = math.log(errs[0] / errs[1], 2)
    assert 3.9 < order < 4.1
    assert errs[1] < 1e-7


def test_heave_constant_force_equilibrium():
    """m h'' + k h = F: starting at the static deflection F/k nothing moves."""
    body = synth.BodyParams(dof=1, m=5.0, k_h=2.0, h0=0.25)
    s = B.initial_state(body)
    for _ in range(50):
        s = B.rk4_step(body, s, 0.5, 0.0, 0.3)
    assert abs(s[0] - 0.25) < 1e-13 and abs(s[2]) < 1e-13


def test_pitch_plunge_normal_mode():
    """2DOF with F = M = 0 started on an eigenvector of (K, M) oscillates in
    that mode at sqrt(lambda)."""
    m, Sa, Ia, kh, ka = 3.0, 0.8, 1.7, 2.0, 5.0
    body = synth.BodyParams(dof=2, m=m, S_a=Sa, I_a=Ia, k_h=kh, k_a=ka)
    Mm = np.array([[m, Sa], [Sa, Ia]])
    K = np.diag([kh, ka])
    lam, V = np.linalg.eig(np.linalg.solve(Mm, K))
    for k in range(2):
        v = V[:, k] / np.max(np.abs(V[:, k])) * 0.1
        w = math.sqrt(lam[k].real)
        s = np.array([v[0].real, v[1].real, 0.0, 0.0])
        dt = 0.01
        for _ in range(500):
            s = B.rk4_step(body, s, 0.0, 0.0, dt)
        t = 500 * dt
        assert s[0] == pytest.approx(v[0].real * math.cos(w * t), abs=1e-9)
        assert s[1] == pytest.approx(v[1].real * math.cos(w * t), abs=1e-9)


def test_heave_nondimensional_form():
    """The lattice parameters satisfy the paper's 1DOF non-dimensional form:
    m* = 4 m / (rho pi D^2) and f_N = sqrt(k/m) / (2 pi) = U / (V_R D)."""
    case = synth.cylinder_viv_case(n_r=8, n_theta=16)
    b = case.bodies[0]
    D, U = case.info["D"], case.info["U"]
    assert 4 * b.m / (math.pi * D * D) == pytest.approx(10.0)
    assert math.sqrt(b.k_h / b.m) / (2 * math.pi) == pytest.approx(U / (5.0 * D))


# ---- Grad wall boundary condition ---------------------------------------------

def channel_grid(ni=16, nj=8):
    jj, ii = np.meshgrid(np.arange(nj, dtype=float), np.arange(ni, dtype=float),
                         indexing="ij")
    return M.Grid(ni, nj, 1, shift_i=(float(ni), 0.0)), ii, jj


@pytest.mark.parametrize("T0", [1.0 / 3.0, 0.25])
def test_grad_wall_populations_carry_navier_stokes_stress(T0):
    """Linear shear u_x = s y over a resting flat wall: the Grad populations
    built at the wall have density rho, zero velocity and the pre-collision
    non-equilibrium shear stress -(dt/omega) p s (Chapman-Enskog), and zero heat
    flux."""
    grid, X, Y = channel_grid()
    gamma, mu, Pr, dt, sr = 1.4, 0.03, 0.71, 0.4, 2e-3
    rho = np.ones_like(X)
    ux = sr * Y
    T = np.full_like(X, T0)
    f, g = L.equilibrium_populations(rho, ux, 0 * X, T, gamma)
    f_old, g_old = f.copy(), g.copy()
    missing = np.zeros(f.shape, dtype=bool)
    missing[:, 0, :] = True
    zero = np.zeros_like(X)
    wall_grad_bc(grid, X, Y, X, Y, zero, zero, f, g, missing, f_old, g_old, gamma, mu,
                 Pr, dt)
    f0, g0 = f[:, 0, :], g[:, 0, :]
    cx = np.array(L.CX, float)[:, None]
    cy = np.array(L.CY, float)[:, None]
    omega = 1 / (mu / (T0 * dt) + 0.5)
    assert np.allclose(f0.sum(0), 1.0, atol=1e-14)
    assert np.allclose((f0 * cx).sum(0), 0.0, atol=1e-15)
    assert np.allclose((f0 * cy).sum(0), 0.0, atol=1e-15)
    assert np.allclose((f0 * cx * cy).sum(0), -(dt / omega) * T0 * sr, rtol=1e-12, atol=0)
    Cv = 1 / (gamma - 1)
    assert np.allclose(g0.sum(0), 2 * Cv * T0, rtol=1e-13)
    assert np.allclose((g0 * cx).sum(0), 0.0, atol=1e-14)
    assert np.allclose((g0 * cy).sum(0), 0.0, atol=1e-14)


def test_grad_wall_moving_wall_and_target_at_B():
    """The wall velocity is imposed (u_t = V_G) and rho_t, T_t come from B at
    distance dt along the normal: for fields linear in y with the wall row
    holding the previous values, the targets are the values at y = dt."""
    grid, X, Y = channel_grid()
    gamma, mu, Pr, dt = 1.4, 0.03, 0.71, 0.4
    rho = 1.0 + 0.01 * Y
    T = 0.3 + 0.004 * Y
    f, g = L.equilibrium_populations(rho, 0 * X, 0 * X, T, gamma)
    missing = np.zeros(f.shape, dtype=bool)
    missing[:, 0, :] = True
    VGx = np.full_like(X, 0.02)
    VGy = np.full_like(X, -0.01)
    rt, uxt, uyt, Tt = wall_grad_bc(grid, X, Y, X, Y, VGx, VGy, f, g, missing,
                                    f.copy(), g.copy(), gamma, mu, Pr, dt)
    assert np.allclose(rt, 1.0 + 0.01 * dt, rtol=1e-13)
    assert np.allclose(Tt, 0.3 + 0.004 * dt, rtol=1e-13)
    f0 = f[:, 0, :]
    cx = np.array(L.CX, float)[:, None]
    cy = np.array(L.CY, float)[:, None]
    assert np.allclose((f0 * cx).sum(0) / f0.sum(0), 0.02, rtol=1e-12)
    assert np.allclose((f0 * cy).sum(0) / f0.sum(0), -0.01, rtol=1e-12)


# ---- P17 / P18: whole coupled steps ---------------------------------------------

def small_cylinder(h0_frac=0.0, **kw):
    return synth.cylinder_viv_case(n_r=24, n_theta=48, D=16.0, first_cell_frac=0.06,
                                   r_far_D=6.0, blend_D=3.0, h0_frac=h0_frac, **kw)


def test_symmetric_cylinder_has_zero_lift():
    """P17: symmetric O-grid, flow along x, no perturbation: C_L stays at
    round-off level and the body does not move."""
    case = small_cylinder()
    s = OracleSolver(case.mesh, case.fluid, case.bodies)
    s.run(25)
    lifts = [abs(h[2]) for h in s.history]
    drags = [h[1] for h in s.history]
    assert max(lifts) < 1e-12 * max(abs(d) for d in drags)
    assert abs(s.states[0][0]) < 1e-12


def test_fixed_body_equivalence():
    """P18: an infinitely heavy spring-mounted body equals a fixed body, bitwise."""
    case = small_cylinder(h0_frac=0.0)
    heavy = synth.configs.replace(case.bodies[0], m=math.inf)
    fixed = synth.configs.replace(case.bodies[0], dof=3)
    fluid = synth.configs.replace(case.fluid, u_inf=(0.1, 0.02))
    a = OracleSolver(case.mesh, fluid, [heavy])
    b = OracleSolver(case.mesh, fluid, [fixed])
    a.run(10)
    b.run(10)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.g, b.g)


def test_moving_cylinder_runs_and_wall_moves_with_body():
    """Coupled run with an initial heave: the body oscillates, the populations
    stay finite and the wall nodes move rigidly with it."""
    case = small_cylinder(h0_frac=0.05, mstar=2.0, ustar=3.0)
    s = OracleSolver(case.mesh, case.fluid, case.bodies)
    s.run(15)
    assert np.all(np.isfinite(s.f)) and np.all(np.isfinite(s.g))
    h = s.states[0][0]
    assert h != case.bodies[0].h0
    x, y = s.positions(s.states)
    assert np.allclose(y[0] - case.mesh.Y[0], h, atol=1e-12)
    assert np.allclose(x[0], case.mesh.X[0], atol=1e-12)
