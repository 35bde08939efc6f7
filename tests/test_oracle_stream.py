"""Pins of the oracle's ALE semi-Lagrangian transport (paper Sec. II.A-B) and
blending-function mesh motion (Sec. II.D): interpolation exactness, the
bilinear inverse map, the exact lattice shift, uniform-flow preservation and
the characteristic foot of the departure point."""

import numpy as np
import pytest

import synth
from oracle import lattice as L
from oracle import mesh as M
from oracle import stream as S
from oracle.solver import OracleSolver


# ---- P6: quadratic Lagrange interpolation ----------------------------------

def test_lagrange_partition_reproduction_kronecker():
    a = np.linspace(-1.0, 1.0, 41)
    Ls = {p: S.lagrange_1d(p, a) for p in (-1, 0, 1)}
    assert np.max(np.abs(sum(Ls.values()) - 1.0)) < 1e-15
    assert np.max(np.abs(sum(p * Ls[p] for p in Ls) - a)) < 1e-15
    assert np.max(np.abs(sum(p * p * Ls[p] for p in Ls) - a * a)) < 1e-15
    for p in (-1, 0, 1):
        for q in (-1, 0, 1):
            assert S.lagrange_1d(p, np.array([float(q)]))[0] == (1.0 if p == q else 0.0)


def test_interpolate_reproduces_biquadratic_fields():
    rng = np.random.default_rng(1)
    mesh = synth.cartesian_mesh(16, 12)
    grid = M.Grid.from_mesh(mesh)
    coef = rng.normal(size=(3, 3))

    def poly(x, y):
        return sum(coef[m, n] * x ** m * y ** n for m in range(3) for n in range(3))

    F = poly(mesh.X, mesh.Y)
    a = rng.uniform(-1, 1, F.shape)
    b = rng.uniform(-1, 1, F.shape)
    out = S.interpolate(grid, F, a, b)
    inner = (slice(2, -2), slice(2, -2))
    ref = poly(mesh.X + a, mesh.Y + b)
    assert np.max(np.abs(out[inner] - ref[inner])) < 1e-11 * np.max(np.abs(ref))


# ---- P7: bilinear inverse ----------------------------------------------------

def test_bilinear_inverse_residual_on_distorted_cells():
    rng = np.random.default_rng(2)
    n = 500
    P00 = (rng.uniform(-0.2, 0.2, n), rng.uniform(-0.2, 0.2, n))
    P10 = (1 + rng.uniform(-0.2, 0.2, n), rng.uniform(-0.2, 0.2, n))
    P01 = (rng.uniform(-0.2, 0.2, n), 1 + rng.uniform(-0.2, 0.2, n))
    P11 = (1 + rng.uniform(-0.2, 0.2, n), 1 + rng.uniform(-0.2, 0.2, n))
    s0 = rng.uniform(0, 1, n)
    t0 = rng.uniform(0, 1, n)
    Px = P00[0] * (1 - s0) * (1 - t0) + P10[0] * s0 * (1 - t0) + P01[0] * (1 - s0) * t0 + P11[0] * s0 * t0
    Py = P00[1] * (1 - s0) * (1 - t0) + P10[1] * s0 * (1 - t0) + P01[1] * (1 - s0) * t0 + P11[1] * s0 * t0
    s, t, res = S.bilinear_inverse(P00, P10, P01, P11, Px, Py)
    assert np.max(res) < 1e-13
    assert np.max(np.abs(s - s0)) < 1e-12 and np.max(np.abs(t - t0)) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_departure_offsets_on_affine_mesh_are_exact(seed):
    """On X = A xi + b the cells are parallelograms, so xi_dp - xi =
    A^{-1}(X_dp - X) exactly, for every velocity."""
    rng = np.random.default_rng(seed)
    A = np.eye(2) + rng.uniform(-0.3, 0.3, (2, 2))
    base = synth.cartesian_mesh(10, 10)
    X = A[0, 0] * base.X + A[0, 1] * base.Y + 3.0
    Y = A[1, 0] * base.X + A[1, 1] * base.Y - 1.0
    grid = M.Grid(10, 10, 0, shift_i=(A[0, 0] * 10, A[1, 0] * 10),
                  shift_j=(A[0, 1] * 10, A[1, 1] * 10))
    dt = rng.uniform(0.2, 0.5)
    Ainv = np.linalg.inv(A)
    chat = S.transformed_velocities(grid, X, Y, X, Y, 0.0 * X, 0.0 * X)
    for i in range(1, 9):
        chx, chy = chat[i]
        # static mesh: c^ = c (g = I)
        assert np.max(np.abs(chx - L.CX[i])) < 1e-14
        assert np.max(np.abs(chy - L.CY[i])) < 1e-14
        a, b, miss = S.departure_offsets(grid, X, Y, chx, chy, dt)
        ea = Ainv[0, 0] * (-dt * L.CX[i]) + Ainv[0, 1] * (-dt * L.CY[i])
        eb = Ainv[1, 0] * (-dt * L.CX[i]) + Ainv[1, 1] * (-dt * L.CY[i])
        assert np.max(np.abs(a - ea)) < 1e-12 and np.max(np.abs(b - eb)) < 1e-12
        assert not miss.any()


def test_departure_exceeding_the_cells_raises():
    mesh = synth.cartesian_mesh(8, 8)
    grid = M.Grid.from_mesh(mesh)
    chx = np.full(mesh.X.shape, 1.0)
    with pytest.raises(S.CFLViolation):
        S.departure_offsets(grid, mesh.X, mesh.Y, chx, 0 * chx, 1.2)


# ---- P8: exact lattice shift ---------------------------------------------

def test_unit_cfl_streaming_is_exact_lattice_shift():
    """Undeformed unit grid, dt = 1, static: streaming is np.roll by c_i, bitwise."""
    rng = np.random.default_rng(4)
    mesh = synth.cartesian_mesh(12, 9)
    grid = M.Grid.from_mesh(mesh)
    fpost = rng.uniform(0.01, 0.5, (9, 9, 12))
    gpost = rng.uniform(0.01, 0.5, (9, 9, 12))
    zero = np.zeros_like(mesh.X)
    f_new, g_new, missing = S.stream(grid, mesh.X, mesh.Y, mesh.X, mesh.Y, zero, zero,
                                     1.0, fpost, gpost)
    for i in range(9):
        ref_f = np.roll(fpost[i], (L.CY[i], L.CX[i]), axis=(0, 1))
        ref_g = np.roll(gpost[i], (L.CY[i], L.CX[i]), axis=(0, 1))
        assert np.array_equal(f_new[i], ref_f), i
        assert np.array_equal(g_new[i], ref_g), i
    assert not missing.any()


# ---- P9: uniform flow preservation ---------------------------------------

@pytest.mark.parametrize("amp,T,moving", [(0.05, 1 / 3, False), (0.35, 0.2, False),
                                          (0.05, 1 / 3, True), (0.3, 0.25, True)])
def test_uniform_flow_preserved_on_deformed_mesh(amp, T, moving):
    mesh = synth.periodic_sine_mesh(32, amp)
    fluid = synth.FluidParams(gamma=1.4, Pr=0.71, mu=0.02, rho_inf=1.0, T_inf=T,
                              u_inf=(0.08, -0.05), dt=0.4)
    bodies = []
    if moving:
        bodies = [synth.BodyParams(dof=0, center=(16.0, 16.0), ea=(16.5, 15.5),
                                   r_rigid=3.0, r_blend=11.0, heave_amp=0.8,
                                   heave_freq=0.01, pitch_amp=0.3, pitch_freq=0.013)]
    rho, ux, uy, TT = synth.configs.uniform_fields(mesh, 1.0, fluid.u_inf, T)
    s = OracleSolver(mesh, fluid, bodies, rho, ux, uy, TT)
    f0, g0 = s.f.copy(), s.g.copy()
    s.run(12)
    assert np.max(np.abs(s.f - f0)) < 1e-13
    assert np.max(np.abs(s.g - g0)) < 1e-13


# ---- P16: blending ---------------------------------------------------------

def test_blending_polynomial_end_conditions():
    assert M.r5(0.0) == 0.0 and M.r5(1.0) == 1.0
    # r5(h) = O(h^3) and 1 - r5(1 - h) = O(h^3): first and second derivatives
    # vanish at both ends
    for h in (1e-2, 1e-3, 1e-4):
        assert abs(M.r5(h)) <= 10.0 * h ** 3 * 1.0001
        assert abs(1.0 - M.r5(1.0 - h)) <= 10.0 * h ** 3 * 1.0001
        assert abs(M.r5(h)) >= 9.0 * h ** 3
    s = np.linspace(0, 1, 101)
    assert np.all(np.diff(M.r5(s)) > 0)
    assert M.r5(0.5) == pytest.approx(0.5)


def test_blended_mesh_rigid_and_identity_zones():
    mesh = synth.ogrid_mesh(40, 80, 20.0, 0.5, 300.0)
    body = synth.BodyParams(dof=2, center=(0.0, 0.0), ea=(3.0, -1.0), r_rigid=15.0,
                            r_blend=120.0)
    h, alpha = 2.5, 0.2
    x, y = M.deformed_positions(mesh.X, mesh.Y, [body], [(h, alpha, 0, 0)])
    d = np.hypot(mesh.X, mesh.Y)
    c, s = np.cos(alpha), np.sin(alpha)
    gx = 3.0 + c * (mesh.X - 3.0) - s * (mesh.Y + 1.0)
    gy = -1.0 + h + s * (mesh.X - 3.0) + c * (mesh.Y + 1.0)
    rigid = d <= 15.0
    assert np.max(np.abs(x[rigid] - gx[rigid])) < 1e-12
    assert np.max(np.abs(y[rigid] - gy[rigid])) < 1e-12
    far = d >= 120.0
    assert np.array_equal(x[far], mesh.X[far]) and np.array_equal(y[far], mesh.Y[far])
    grid = M.Grid.from_mesh(mesh)
    x_xi, x_eta, y_xi, y_eta = grid.metrics(x, y)
    assert np.all(x_xi * y_eta - y_xi * x_eta > 0)


# ---- P19: ALE transformed velocity and characteristic foot -------------------

def test_transformed_velocity_closed_forms():
    """c^ = A^{-1}(c - V) for an affine motion x = A X + b of a curvilinear mesh
    (the FE metrics are exact on affine maps); checked away from the seams."""
    rng = np.random.default_rng(5)
    mesh = synth.periodic_sine_mesh(16, 0.2)
    grid = M.Grid(16, 16, 1)          # interior nodes never touch a seam
    A = np.array([[np.cos(0.7), -np.sin(0.7)], [np.sin(0.7), np.cos(0.7)]]) @ \
        np.array([[1.1, 0.2], [0.0, 0.9]])
    x1 = A[0, 0] * mesh.X + A[0, 1] * mesh.Y + 5.0
    y1 = A[1, 0] * mesh.X + A[1, 1] * mesh.Y - 2.0
    V = rng.normal(size=2) * 0.1
    chat = S.transformed_velocities(grid, mesh.X, mesh.Y, x1, y1,
                                    V[0] + 0 * x1, V[1] + 0 * x1)
    Ainv = np.linalg.inv(A)
    inner = (slice(2, -2), slice(2, -2))
    for i in range(9):
        ex = Ainv @ np.array([L.CX[i] - V[0], L.CY[i] - V[1]])
        assert np.max(np.abs(chat[i][0][inner] - ex[0])) < 1e-12
        assert np.max(np.abs(chat[i][1][inner] - ex[1])) < 1e-12


def characteristic_foot_residual(alpha_n, alpha_n1, b_n, b_n1, dt=0.5, transpose=False):
    """|x^n(X_dp) - (x^{n+1}(X) - c dt)| over the interior, for a rigid motion."""
    mesh = synth.cartesian_mesh(20, 20)
    grid = M.Grid(20, 20, 1)   # non-periodic j, periodic i unused inside
    X, Y = mesh.X, mesh.Y

    def rigid(al, b):
        c, s = np.cos(al), np.sin(al)
        return c * X - s * Y + b[0], s * X + c * Y + b[1]

    x0, y0 = rigid(alpha_n, b_n)
    x1, y1 = rigid(alpha_n1, b_n1)
    VGx, VGy = (x1 - x0) / dt, (y1 - y0) / dt
    chat = S.transformed_velocities(grid, X, Y, x1, y1, VGx, VGy)
    worst = 0.0
    inner = (slice(3, -3), slice(3, -3))
    for i in range(1, 9):
        chx, chy = chat[i]
        if transpose:   # planted mistake: g^T in place of g^{-1}
            c1, s1 = np.cos(alpha_n1), np.sin(alpha_n1)
            wx, wy = L.CX[i] - VGx, L.CY[i] - VGy
            chx, chy = c1 * wx - s1 * wy, s1 * wx + c1 * wy
        Xdp = X - dt * chx
        Ydp = Y - dt * chy
        c, s = np.cos(alpha_n), np.sin(alpha_n)
        xf = c * Xdp - s * Ydp + b_n[0]
        yf = s * Xdp + c * Ydp + b_n[1]
        r = np.hypot(xf - (x1 - dt * L.CX[i]), yf - (y1 - dt * L.CY[i]))
        worst = max(worst, float(np.max(r[inner])))
    return worst


def test_departure_is_characteristic_foot_for_translation():
    assert characteristic_foot_residual(0.0, 0.0, (0.3, -0.2), (0.37, -0.11)) < 1e-13


def test_departure_foot_first_order_in_rotation_increment():
    dal = 2e-4
    r = characteristic_foot_residual(0.5, 0.5 + dal, (0.1, 0.0), (0.12, 0.01))
    assert r < 3.0 * 0.5 * dal * 2.0          # dt |d alpha| |c - V_G| bound
    # the transposed Jacobian would be off by an O(alpha) rotation of c
    wrong = characteristic_foot_residual(0.5, 0.5 + dal, (0.1, 0.0), (0.12, 0.01),
                                         transpose=True)
    assert wrong > 100 * r
