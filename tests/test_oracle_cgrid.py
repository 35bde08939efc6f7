"""Oracle pins for the C-grid topology: the mirror map across the wake cut,
index-space derivatives, far-field node set, force closure, the rest state,
and mirror symmetry of the flow past a symmetric section at zero incidence
(a wrong mirror index or a one-sided rule in the wrong place breaks it)."""

from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import forces as FO
from oracle import lattice as L
from oracle.boundary import farfield_nodes
from oracle.mesh import Grid
from oracle.solver import OracleSolver
from oracle.stream import boundary_nodes, stencil_centres

DOF_FIXED = 3


def small(**kw):
    args = dict(n_wake=16, n_af=64, nj=32, chord=40.0, first_cell=0.5, far_chords=4.0)
    args.update(kw)
    return synth.cgrid_mesh(**args)


def test_mesh_layout_and_duplicates():
    m = small()
    assert (m.ni, m.nj, m.n_wake) == (96, 32, 16)
    nw = m.n_wake
    # cut nodes and the trailing edge appear twice on row 0
    for i in range(nw + 1):
        assert m.X[0, i] == m.X[0, m.ni - 1 - i] and m.Y[0, i] == m.Y[0, m.ni - 1 - i]
    assert m.X[0, nw] == 40.0 and m.Y[0, nw] == 0.0
    # section: thickness 0.12 c at 0.3 c (NACA 0012), closed trailing edge
    ya = m.Y[0, nw:m.ni - nw]
    assert 0.11 * 40 < ya.max() - ya.min() < 0.125 * 40
    # right-handed in (i, j) everywhere (centred / one-sided differences)
    g = Grid.from_mesh(m)
    x_xi, x_eta, y_xi, y_eta = g.metrics(m.X, m.Y)
    assert np.all(x_xi * y_eta - y_xi * x_eta > 0)


def test_mirror_map_continues_each_cut_column():
    """Node (i, -1) of a cut column is (ni-1-i, 1): it must continue column
    i smoothly across the cut (quadratic extrapolation from rows 0..2 lands
    close to it), and no other node of the upper side does."""
    m = small()
    g = Grid.from_mesh(m)
    nw = m.n_wake
    for i in list(range(1, nw)) + list(range(m.ni - nw, m.ni - 1)):
        si, sj, ok = g.node_index(i, -1)
        assert ok and (int(si), int(sj)) == (m.ni - 1 - i, 1)
        ex = 3 * m.X[0, i] - 3 * m.X[1, i] + m.X[2, i]
        ey = 3 * m.Y[0, i] - 3 * m.Y[1, i] + m.Y[2, i]
        d = np.hypot(m.X[1] - ex, m.Y[1] - ey)
        assert int(np.argmin(d)) == m.ni - 1 - i
        assert d.min() < 0.2 * np.hypot(m.X[1, i] - m.X[0, i], m.Y[1, i] - m.Y[0, i])
    # exit columns have no neighbour beyond them
    assert not g.node_index(-1, 3)[2] and not g.node_index(m.ni, 3)[2]


def test_linear_field_gradient_is_exact_everywhere():
    m = small()
    g = Grid.from_mesh(m)
    C = 0.3 * m.X - 0.7 * m.Y + 2.0
    gx, gy = g.grad(C, m.X, m.Y)
    assert np.max(np.abs(gx - 0.3)) < 1e-10 and np.max(np.abs(gy + 0.7)) < 1e-10


def test_derivative_across_the_cut_is_centred():
    """d/dj at a cut node uses row 1 of both sides: for a field that is odd
    across the chord line (C = y) the centred difference equals the mean of
    the two one-sided rows, and differs from the one-sided wall formula."""
    m = small()
    g = Grid.from_mesh(m)
    dj = g.d_j(m.Y)
    i = 5
    assert dj[0, i] == pytest.approx(0.5 * (m.Y[1, i] - m.Y[1, m.ni - 1 - i]), rel=1e-14)
    one_sided = 0.5 * (-3 * m.Y[0, i] + 4 * m.Y[1, i] - m.Y[2, i])
    assert abs(dj[0, i] - one_sided) > 1e-3 * abs(dj[0, i])
    # wall columns stay one-sided
    k = m.n_wake + 10
    assert dj[0, k] == pytest.approx(0.5 * (-3 * m.Y[0, k] + 4 * m.Y[1, k] - m.Y[2, k]), rel=1e-14)


def test_far_field_nodes_and_stencil_centres():
    m = small()
    g = Grid.from_mesh(m)
    far = boundary_nodes(g)
    assert far.sum() == m.ni + 2 * (m.nj - 1)
    jj, ii, nx, ny, jr, ir = farfield_nodes(g, m.X, m.Y)
    assert len(jj) == far.sum() and np.all(far[jj, ii])
    assert not np.any(far[jr, ir])                  # outlets copy interior nodes
    # outward normals: upstream row points to -x, exit columns to +x
    up = (jj == m.nj - 1) & (ii == m.ni // 2)
    assert nx[up][0] < 0
    ex = (ii == 0) & (jj == m.nj // 2)
    assert nx[ex][0] > 0 and nx[(ii == m.ni - 1) & (jj == m.nj // 2)][0] > 0
    ic, jc = stencil_centres(g)
    assert jc[0, 3] == 0 and jc[0, m.n_wake] == 1 and np.all(ic[:, 0] == 1)


def test_uniform_pressure_gives_zero_force_and_moment():
    m = small()
    g = Grid.from_mesh(m)
    shape = m.X.shape
    rho = np.full(shape, 1.3)
    f, gg = L.equilibrium_populations(rho, np.zeros(shape), np.zeros(shape),
                                      np.full(shape, 0.3), 1.4)
    Fx, Fy, M = FO.wall_force(g, f, gg, m.X, m.Y, 1.4, 0.01, 0.71, 0.1, (10.0, 0.0))
    scale = 1.3 * 0.3 * 2.1 * 40.0
    assert abs(Fx) < 1e-13 * scale and abs(Fy) < 1e-13 * scale and abs(M) < 1e-11 * scale * 40


def test_rest_state_is_preserved_with_a_fixed_section():
    c = synth.small_airfoil_case(alpha0_deg=0.0)
    body = replace(c.bodies[0], dof=DOF_FIXED)
    fl = replace(c.fluid, u_inf=(0.0, 0.0))
    ora = OracleSolver(c.mesh, fl, [body])
    f0, g0 = ora.f.copy(), ora.g.copy()
    ora.run(20)
    assert np.max(np.abs(ora.f - f0)) < 1e-13 and np.max(np.abs(ora.g - g0)) < 1e-13


@pytest.mark.slow
def test_flow_past_symmetric_section_stays_mirror_symmetric():
    c = synth.small_airfoil_case(alpha0_deg=0.0)
    body = replace(c.bodies[0], dof=DOF_FIXED)
    ora = OracleSolver(c.mesh, c.fluid, [body], c.rho, c.ux, c.uy, c.T)
    ora.run(40)
    rho, ux, uy, _, T = ora.macroscopic()
    mir = slice(None, None, -1)
    assert np.max(np.abs(rho - rho[:, mir])) < 1e-11
    assert np.max(np.abs(ux - ux[:, mir])) < 1e-11
    assert np.max(np.abs(uy + uy[:, mir])) < 1e-11
    # the flow has developed (not a trivially symmetric rest state)
    assert np.max(np.abs(uy)) > 1e-3
    h = np.array(ora.history)
    assert np.max(np.abs(h[:, 2])) < 1e-9 * np.max(np.abs(h[:, 1]))
