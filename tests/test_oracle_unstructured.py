"""Oracle pins for the step on unstructured 9-node quadrilateral meshes: the
mesh itself, the element shape functions, finite-element gradients (exact for
linear fields on the deformed mesh), point location in the patch of a node,
the rest state, and the shear-wave decay rate nu k^2 with nu = mu / rho (the
viscosity the collision sets), which a wrong element, stencil or gradient
would change."""

import numpy as np
import pytest

from oracle import lattice as L
from oracle.unstructured import LOCAL, UGrid, UnstructuredSolver, bilinear_local, shape
from synth.configs import FluidParams
from synth.unstructured import (element_coords, smallest_patch_reach, unstructured_pulse_case,
                                unstructured_q9_mesh)


@pytest.fixture(scope="module")
def mesh():
    return unstructured_q9_mesh(8, amp=0.06, seed=3)


@pytest.fixture(scope="module")
def grid(mesh):
    return UGrid(mesh)


def test_mesh_is_unstructured_straight_sided_and_valid(mesh, grid):
    ex, ey = element_coords(mesh)
    Lx, Ly = mesh.period
    # the elements tile the periodic box
    x, y = ex[:, :4], ey[:, :4]
    area = 0.5 * np.sum(x * np.roll(y, -1, axis=1) - np.roll(x, -1, axis=1) * y, axis=1)
    assert np.all(area > 0) and abs(area.sum() - Lx * Ly) < 1e-9 * Lx * Ly
    # edge and centre nodes where the corners' bilinear map puts them
    for k, (a, b) in enumerate(((0, 1), (1, 2), (2, 3), (3, 0))):
        assert np.max(np.abs(ex[:, 4 + k] - 0.5 * (ex[:, a] + ex[:, b]))) < 1e-12
    assert np.max(np.abs(ey[:, 8] - ey[:, :4].mean(axis=1))) < 1e-12
    # irregular vertices: 3 and 5 or more elements meet at some corners
    counts = np.bincount(mesh.elems.ravel(), minlength=mesh.n_nodes)
    assert np.any(counts == 3) and np.any(counts >= 5)
    # positive Jacobian of the 9-node map at every element node
    assert np.all(np.isfinite(grid.Wx))
    for a in range(9):
        from oracle.unstructured import shape_grad
        dxi, deta = shape_grad(np.array(LOCAL[a, 0]), np.array(LOCAL[a, 1]))
        det = (ex @ dxi) * (ey @ deta) - (ey @ dxi) * (ex @ deta)
        assert np.all(det > 0)


def test_shape_functions():
    rng = np.random.default_rng(0)
    xi, eta = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50)
    N = shape(xi, eta)
    assert np.max(np.abs(N.sum(axis=0) - 1)) < 1e-14
    # Kronecker at the nodes
    Nn = shape(LOCAL[:, 0], LOCAL[:, 1])
    assert np.max(np.abs(Nn - np.eye(9))) < 1e-15
    # biquadratic polynomials are reproduced
    for p in range(3):
        for q in range(3):
            vals = LOCAL[:, 0] ** p * LOCAL[:, 1] ** q
            assert np.max(np.abs(vals @ N - xi ** p * eta ** q)) < 1e-13


def test_gradients_of_linear_fields_are_exact(mesh, grid):
    Lx = mesh.period[0]
    for (a, b) in ((0.3, -0.7), (1.0, 0.0), (-0.2, 0.45)):
        # a linear field of the unwrapped coordinates: constant gradient
        # everywhere except across the periodic seam, which element derivatives
        # never straddle (each element uses its own unwrapped coordinates)
        Ce = a * grid.ex + b * grid.ey
        gx_e = np.einsum("eas,es->ea", grid.Wx, Ce)
        gy_e = np.einsum("eas,es->ea", grid.Wy, Ce)
        assert np.max(np.abs(gx_e - a)) < 1e-11 and np.max(np.abs(gy_e - b)) < 1e-11
    # nodal recovery of a smooth periodic field converges (second order)
    errs = []
    for m in (4, 8):
        me = unstructured_q9_mesh(m, amp=0.06, seed=3)
        g = UGrid(me)
        k = 2 * np.pi / me.period[0]
        gx, gy = g.grad(np.sin(k * me.X) * np.cos(k * me.Y))
        ex = k * np.cos(k * me.X) * np.cos(k * me.Y)
        errs.append(np.max(np.abs(gx - ex)) / k)
    assert errs[1] < errs[0] / 3.0


def test_point_location_in_the_patch(mesh, grid):
    rng = np.random.default_rng(1)
    r = smallest_patch_reach(mesh)
    for _ in range(4):
        ang = rng.uniform(0, 2 * np.pi)
        rad = rng.uniform(0, 0.9 * r)
        dx, dy = rad * np.cos(ang), rad * np.sin(ang)
        e, xi, eta = grid.locate(np.full(grid.N, dx), np.full(grid.N, dy))
        assert np.all(np.abs(xi) <= 1 + 1e-12) and np.all(np.abs(eta) <= 1 + 1e-12)
        # the bilinear map of the element takes (xi, eta) to the point
        n = np.arange(grid.N)
        a = grid.pa[n, np.argmax((grid.pe == e[:, None]) & grid.pm, axis=1)]
        px = grid.ex[e, a] + dx
        py = grid.ey[e, a] + dy
        cx, cy = grid.ex[e, :4], grid.ey[e, :4]
        w = [(1 - xi) * (1 - eta) / 4, (1 + xi) * (1 - eta) / 4, (1 + xi) * (1 + eta) / 4,
             (1 - xi) * (1 + eta) / 4]
        rx = sum(w[c] * cx[:, c] for c in range(4)) - px
        ry = sum(w[c] * cy[:, c] for c in range(4)) - py
        assert np.max(np.hypot(rx, ry)) < 1e-11
    # zero displacement finds each node at its own local position: the
    # interpolation returns the nodal value
    e, xi, eta = grid.locate(np.zeros(grid.N), np.zeros(grid.N))
    f = np.random.default_rng(2).standard_normal(grid.N)
    val = np.sum(shape(xi, eta).T * f[grid.elems[e]], axis=1)
    assert np.max(np.abs(val - f)) < 1e-12
    with pytest.raises(ValueError):
        grid.locate(np.full(grid.N, 10.0 * mesh.period[0] / 8), np.zeros(grid.N))


def test_bilinear_local_inverts_the_map():
    rng = np.random.default_rng(4)
    cx = np.array([[0.0, 2.0, 2.3, -0.2]])
    cy = np.array([[0.0, 0.1, 1.9, 1.6]])
    xi0, eta0 = rng.uniform(-1, 1, 2)
    w = [(1 - xi0) * (1 - eta0) / 4, (1 + xi0) * (1 - eta0) / 4, (1 + xi0) * (1 + eta0) / 4,
         (1 - xi0) * (1 + eta0) / 4]
    px = np.array([sum(w[c] * cx[0, c] for c in range(4))])
    py = np.array([sum(w[c] * cy[0, c] for c in range(4))])
    xi, eta = bilinear_local(cx, cy, px, py)
    assert abs(xi[0] - xi0) < 1e-13 and abs(eta[0] - eta0) < 1e-13


def test_rest_state_and_uniform_stream_are_preserved(mesh):
    N = mesh.n_nodes
    dt = smallest_patch_reach(mesh) / (3 * np.sqrt(2))
    fl = FluidParams(gamma=1.4, Pr=0.71, mu=0.02, rho_inf=1.0, T_inf=0.3, u_inf=(0.04, -0.03),
                     dt=dt)
    o = UnstructuredSolver(mesh, fl)
    f0, g0 = o.f.copy(), o.g.copy()
    o.run(50)
    assert np.max(np.abs(o.f - f0)) < 1e-13 and np.max(np.abs(o.g - g0)) < 1e-13


def test_shear_wave_decays_at_the_viscous_rate(mesh):
    Lx = mesh.period[0]
    dt = smallest_patch_reach(mesh) / (3 * np.sqrt(2))
    mu = 0.05
    fl = FluidParams(gamma=1.4, Pr=0.71, mu=mu, rho_inf=1.0, T_inf=1 / 3, u_inf=(0, 0), dt=dt)
    k = 2 * np.pi / Lx
    N = mesh.n_nodes
    o = UnstructuredSolver(mesh, fl, np.ones(N), 1e-3 * np.sin(k * mesh.Y), np.zeros(N),
                           np.full(N, 1 / 3))

    def amplitude():
        _, u, _, _, _ = o.macroscopic()
        return 2 * np.mean(u * np.sin(k * mesh.Y))

    a0 = amplitude()
    n = 800
    o.run(n)
    rate = -np.log(amplitude() / a0) / (n * dt)
    assert abs(rate / (mu * k * k) - 1) < 0.03


def test_pulse_case_runs():
    mesh, fl, (rho, ux, uy, T) = unstructured_pulse_case(4)
    o = UnstructuredSolver(mesh, fl, rho, ux, uy, T)
    m0 = rho.sum()
    o.run(10)
    r, _, _, _, _ = o.macroscopic()
    assert np.all(np.isfinite(r)) and abs(r.sum() - m0) < 1e-6 * m0
