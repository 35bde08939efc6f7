"""Oracle pins for the step on an unstructured 9-node mesh round a fixed
cylinder: the mesh (annulus tiled, wall and far-field nodes on their
polygons, clockwise wall), missing populations at the wall exactly those
arriving from inside the body, the points B, gas at rest kept at rest with
zero force, and exact mirror symmetry (zero lift) of the flow past the body
on a mesh that is its own mirror image."""

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import lattice as L
from oracle.unstructured import UGrid, UnstructuredWallSolver, shape
from synth.configs import BodyParams, FluidParams
from synth.unstructured import (cylinder_q9_mesh, element_coords, q9_cylinder_case,
                                smallest_patch_reach)


@pytest.fixture(scope="module")
def mesh():
    return cylinder_q9_mesh(32, 40.0, 6.0, seed=1)


def polygon_area(x, y):
    return 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)


def test_annulus_mesh(mesh):
    ex, ey = element_coords(mesh)
    x, y = ex[:, :4], ey[:, :4]
    area = 0.5 * np.sum(x * np.roll(y, -1, axis=1) - np.roll(x, -1, axis=1) * y, axis=1)
    assert np.all(area > 0)
    w, f = mesh.wall_nodes, mesh.far_nodes
    # the wall polygon is clockwise, the elements tile the region between it
    # and the outer polygon
    aw = polygon_area(mesh.X[w], mesh.Y[w])
    order = np.argsort(np.arctan2(mesh.Y[f], mesh.X[f]))
    af = polygon_area(mesh.X[f][order], mesh.Y[f][order])
    assert aw < 0
    assert abs(area.sum() - (af + aw)) < 1e-9 * af
    # wall nodes on the chords between the grid's wall points (radius R)
    R = 20.0
    r = np.hypot(mesh.X[w], mesh.Y[w])
    assert np.max(r) <= R + 1e-12 and np.min(r) > R * np.cos(np.pi / 32) - 1e-12
    # every boundary edge of the mesh joins two wall or two far-field nodes
    edges = {}
    for e in mesh.elems:
        for a, b, m in ((0, 1, 4), (1, 2, 5), (2, 3, 6), (3, 0, 7)):
            k = (min(e[a], e[b]), max(e[a], e[b]))
            edges[k] = edges.get(k, 0) + 1
    bnd = set(w.tolist()) | set(f.tolist())
    for (a, b), c in edges.items():
        if c == 1:
            assert a in bnd and b in bnd
    assert len(set(w.tolist()) & set(f.tolist())) == 0


def test_missing_populations_come_from_inside_the_body(mesh):
    dt = smallest_patch_reach(mesh) / (3 * np.sqrt(2))
    fl = FluidParams(gamma=1.4, Pr=0.71, mu=0.05, rho_inf=1.0, T_inf=1 / 3, u_inf=(0, 0), dt=dt)
    o = UnstructuredWallSolver(mesh, fl, BodyParams(dof=3))
    w = o.wall
    wall_set = np.zeros(o.grid.N, dtype=bool)
    wall_set[w] = True
    bnd = wall_set.copy()
    bnd[o.far] = True
    # chord-interior wall nodes (not on the circle): missing exactly when the
    # direction points out of the body, c . n > 0
    on_chord = np.hypot(mesh.X[w], mesh.Y[w]) < 20.0 - 1e-9
    nx, ny = o.nds_x / np.hypot(o.nds_x, o.nds_y), o.nds_y / np.hypot(o.nds_x, o.nds_y)
    checked = 0
    for i in range(1, L.Q):
        miss = o.missing(i)
        assert not np.any(miss & ~bnd)
        cn = L.CX[i] * nx + L.CY[i] * ny
        sel = on_chord & (np.abs(cn) > 1e-6)
        assert np.array_equal(miss[w][sel], cn[sel] > 0)
        checked += sel.sum()
    assert checked > 100


def test_points_B_are_located(mesh):
    dt = smallest_patch_reach(mesh) / (3 * np.sqrt(2))
    fl = FluidParams(gamma=1.4, Pr=0.71, mu=0.05, rho_inf=1.0, T_inf=1 / 3, u_inf=(0, 0), dt=dt)
    o = UnstructuredWallSolver(mesh, fl, BodyParams(dof=3))
    e, xi, eta = o.B
    assert np.all(e >= 0) and np.all(np.abs(xi) <= 1 + 1e-12) and np.all(np.abs(eta) <= 1 + 1e-12)
    nn = np.hypot(o.nds_x, o.nds_y)
    Bx = o.xw + dt * o.nds_x / nn
    By = o.yw + dt * o.nds_y / nn
    # the 9-node map (exact for the straight-sided elements) returns B
    N = shape(xi, eta)
    ex, ey = element_coords(mesh)
    assert np.max(np.abs(np.sum(N.T * ex[e], axis=1) - Bx)) < 1e-10
    assert np.max(np.abs(np.sum(N.T * ey[e], axis=1) - By)) < 1e-10


def test_gas_at_rest_stays_at_rest_with_zero_force(mesh):
    dt = smallest_patch_reach(mesh) / (3 * np.sqrt(2))
    fl = FluidParams(gamma=1.4, Pr=0.71, mu=0.05, rho_inf=1.0, T_inf=1 / 3, u_inf=(0, 0), dt=dt)
    o = UnstructuredWallSolver(mesh, fl, BodyParams(dof=3))
    f0, g0 = o.f.copy(), o.g.copy()
    o.run(20)
    assert np.max(np.abs(o.f - f0)) < 1e-13 and np.max(np.abs(o.g - g0)) < 1e-13
    h = np.array(o.history)
    scale = (1 / 3) * np.pi * 40.0
    assert np.max(np.abs(h[:, 1:4])) < 1e-12 * scale * 20.0


def test_flow_past_the_body_is_mirror_symmetric_with_zero_lift():
    m, fl, b, (rho, ux, uy, T) = q9_cylinder_case(mirror=True)
    _, mm = cKDTree(np.c_[m.X, m.Y]).query(np.c_[m.X, -m.Y])
    o = UnstructuredWallSolver(m, fl, b, rho, ux, uy, T)
    o.run(100)
    r, u, v, E, Tt = o.macroscopic()
    assert np.max(np.abs(r - r[mm])) < 1e-12 and np.max(np.abs(v + v[mm])) < 1e-12
    h = np.array(o.history)
    assert h[-1, 1] > 0.1                              # drag in the stream
    assert np.max(np.abs(h[:, 2])) < 1e-11 * h[-1, 1]  # no lift
    # a developed, non-uniform flow
    assert np.max(np.abs(r - 1.0)) > 1e-4


def test_moving_body_departures_in_the_rigid_zone():
    """A heaving body on the blended unstructured mesh: in the rigid zone
    (r = 0) the mesh translates with the body, g = dx/dX = I and the
    departure point in the undeformed frame is X - dt (c_i - V_G) with
    V_G = (h^{n+1} - h^n) / dt along y, for the rest populations (c_0 = 0)
    too; the located element and local coordinates map back to that point.
    A wall node's rest population is missing exactly where the wall moves
    towards the fluid side of the node (its point X + dt V_G lies in the
    body)."""
    from synth.unstructured import q9_heave_case
    m, fl, b, (r, u, v, T) = q9_heave_case(16, 20.0, 4.0)
    o = UnstructuredWallSolver(m, fl, b, r, u, v, T)
    h0 = o.state[0]
    o.step()
    h1 = o.state[0]
    vg = (h1 - h0) / fl.dt
    assert abs(vg) > 1e-3
    # nodes whose elements lie wholly in the rigid zone (their nodal
    # derivative sees no blending)
    rel = np.all(o.r[m.elems] == 0.0, axis=1)
    g = o.grid
    rigid = np.all(np.where(g.pm, rel[g.pe], True), axis=1)
    ex, ey = element_coords(m)
    checked = 0
    for i in range(L.Q):
        e, xi, eta = o.dep[i]
        ok = rigid & (e >= 0)
        Nw = shape(xi[ok], eta[ok])
        px = np.sum(Nw.T * ex[e[ok]], axis=1)
        py = np.sum(Nw.T * ey[e[ok]], axis=1)
        assert np.max(np.abs(px - (m.X[ok] - fl.dt * L.CX[i]))) < 1e-10
        assert np.max(np.abs(py - (m.Y[ok] - fl.dt * (L.CY[i] - vg)))) < 1e-10
        checked += ok.sum()
    assert checked > 500
    # rest populations at the wall: missing where n . V_G < 0 (n into the fluid)
    nvg = o.nds_y / np.hypot(o.nds_x, o.nds_y) * vg
    miss0 = o.missing(0)[o.wall]
    assert np.all(miss0[nvg < -0.1 * abs(vg)]) and not np.any(miss0[nvg > 0.0])
    assert miss0.sum() > 0.3 * miss0.size


def test_heaving_body_flow_is_mirror_symmetric():
    """A cylinder heaving along y in gas at rest, on a mesh that is its own
    mirror image about the y axis: the flow stays mirror-symmetric and the
    force along x vanishes, while the body feels a force along y."""
    from synth.unstructured import q9_heave_case
    m, fl, b, (r, u, v, T) = q9_heave_case(16, 20.0, 4.0, symmetric=True)
    _, mm = cKDTree(np.c_[m.X, m.Y]).query(np.c_[-m.X, m.Y])
    o = UnstructuredWallSolver(m, fl, b, r, u, v, T)
    o.run(40)
    rr, ux, uy, E, Tt = o.macroscopic()
    assert np.max(np.abs(rr - rr[mm])) < 1e-12 and np.max(np.abs(ux + ux[mm])) < 1e-12
    assert np.max(np.abs(uy - uy[mm])) < 1e-12
    h = np.array(o.history)
    assert abs(h[-1, 2]) > 0.1 and h[-1, 4] != 0.0
    assert np.max(np.abs(h[:, 1])) < 1e-11 * abs(h[-1, 2])


def test_distance_blending_measures_from_the_wall_polygon():
    """Distance blending (Sec. II.D's variant for slender bodies) on the
    cylinder mesh: the wall polygon is the n-gon through the wall points on
    the circle, so the distance of an outside node to it lies between its
    radial distance to the circle and that plus the polygon's sagitta
    R (1 - cos(pi / n)); the blending factor, monotone in the distance, lies
    between the factors of those two distances, and is 0 on the wall."""
    from oracle.mesh import r5
    from synth.unstructured import q9_heave_case
    m, fl, b, (r, u, v, T) = q9_heave_case(16, 20.0, 4.0, distance_blend=True)
    sol = UnstructuredWallSolver(m, fl, b, r, u, v, T)
    R = 10.0
    n = 16
    sag = R * (1.0 - np.cos(np.pi / n))
    d_rad = np.hypot(m.X, m.Y) - R

    def factor(d):
        s = (d - b.r_rigid) / (b.r_blend - b.r_rigid)
        return np.where(s < 0.0, 0.0, np.where(s > 1.0, 1.0, r5(np.clip(s, 0.0, 1.0))))

    assert np.all(sol.r >= factor(d_rad) - 1e-12)
    assert np.all(sol.r <= factor(d_rad + sag) + 1e-12)
    assert np.all(sol.r[m.wall_nodes] == 0.0)
    # the band is narrow against the blending width: the two readings differ
    assert sag < 0.05 * (b.r_blend - b.r_rigid)
    assert np.max(np.abs(sol.r - factor(d_rad))) > 0.0


def test_body_carried_by_uniform_gas_changes_nothing_but_its_position():
    """Galilean check of the moving mesh: a body moving with gas in uniform
    motion (the wall's mesh velocity equals the gas velocity) leaves the gas
    uniform to rounding and feels no force; the wall condition of a fixed body
    (u_t = 0) or a wrong sign of V_G would disturb it at the first step."""
    from synth.unstructured import q9_comoving_case
    m, fl, b, (r, u, v, T) = q9_comoving_case()
    o = UnstructuredWallSolver(m, fl, b, r, u, v, T)
    o.run(30)
    rr, ux, uy, E, Tt = o.macroscopic()
    U = v[0]
    assert np.max(np.abs(rr - 1.0)) < 1e-13 and np.max(np.abs(ux)) < 1e-13
    assert np.max(np.abs(uy - U)) < 1e-13 and np.max(np.abs(Tt - T[0])) < 1e-13
    h = np.array(o.history)
    assert np.max(np.abs(h[:, 1:4])) < 1e-11
    assert abs(h[-1, 4] - 29 * fl.dt * U) < 1e-12


def test_strong_coupling_on_the_unstructured_mesh():
    """Sub-iterations on the moving unstructured mesh: a prescribed body is
    untouched by them (every pass streams onto the same mesh: bitwise the
    staggered step), and for a body on a spring the remaining change of the
    body estimate contracts by 1e3 within three passes."""
    from synth.unstructured import q9_heave_case
    m, fl, b, (r, u, v, T) = q9_heave_case(16, 20.0, 4.0)
    a = UnstructuredWallSolver(m, fl, b, r, u, v, T)
    c = UnstructuredWallSolver(m, fl, b, r, u, v, T)
    c.coupling(3, 0.7)
    a.run(3)
    c.run(3)
    assert np.array_equal(a.f, c.f) and np.array_equal(a.g, c.g)
    m, fl, b, (r, u, v, T) = q9_heave_case(16, 20.0, 4.0, dof=1, mstar=0.5)
    o = UnstructuredWallSolver(m, fl, b, r, u, v, T)
    o.coupling(4, 1.0)
    o.run(3)
    assert o.residuals[0] > 0 and o.residuals[2] < 1e-3 * o.residuals[0]
