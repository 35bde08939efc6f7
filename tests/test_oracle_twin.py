"""Oracle pins for several bodies on the twin O-grid (two cylinders joined by
a slit): the mesh and its mirror map, the wall segments, force closure per
body, exclusive regions of influence, and three symmetries of the flow that a
wrong mirror index, junction merge, segment bound or load sum breaks:

* mirror symmetry about the axis through both cylinders (a stream along it,
  bodies held),
* mirror symmetry about the perpendicular bisector (gas at rest, both
  cylinders released from the same offset),
* under that symmetry a linked pair (one equation, mass m and stiffness k,
  both loads) moves exactly as two independent cylinders of m/2 and k/2 do.
"""

from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import forces as FO
from oracle import lattice as L
from oracle.mesh import Grid, blend_factors, deformed_positions, rigid_map
from oracle.solver import OracleSolver
from oracle.stream import boundary_nodes, stencil_centres

DOF_FIXED = 3
# velocity index under y -> -y and under x -> -x (D2Q9 order of the lattice)
REFLECT_Y = [0, 1, 4, 3, 2, 8, 7, 6, 5]
REFLECT_X = [0, 3, 2, 1, 4, 6, 5, 8, 7]


def small_mesh(**kw):
    args = dict(n_wall=48, n_slit=30, nj=40, diameter=30.0, spacing=90.0, first_cell=0.5,
                far_diameters=8.0)
    args.update(kw)
    return synth.twin_mesh(**args)


def test_mesh_geometry_and_symmetry():
    m = small_mesh()
    nA, s, nB = 48, 30, 48
    assert (m.ni, m.nj, m.n_wake, m.n_wall2) == (nA + 2 * s + nB, 40, s, nB)
    ni = m.ni
    # walls on the circles, slit on the axis between them
    rA = np.hypot(m.X[0, :nA + 1] + 45.0, m.Y[0, :nA + 1])
    rB = np.hypot(m.X[0, nA + s:nA + s + nB + 1] - 45.0, m.Y[0, nA + s:nA + s + nB + 1])
    assert np.max(np.abs(rA - 15.0)) < 1e-12 and np.max(np.abs(rB - 15.0)) < 1e-12
    slit = np.r_[nA:nA + s + 1, nA + s + nB:ni]
    assert np.all(m.Y[0, slit] == 0.0) and np.all(np.abs(m.X[0, slit]) <= 30.0)
    # exact mirror images
    cols = np.arange(ni)
    my, mx = (nA - cols) % ni, (nA + s + nB - cols) % ni
    assert np.array_equal(m.X[:, my], m.X) and np.array_equal(m.Y[:, my], -m.Y)
    assert np.array_equal(m.X[:, mx], -m.X) and np.array_equal(m.Y[:, mx], m.Y)
    # right-handed in (i, j) with the FE metric of the topology; first cells
    g = Grid.from_mesh(m)
    x_xi, x_eta, y_xi, y_eta = g.metrics(m.X, m.Y)
    assert np.all(x_xi * y_eta - y_xi * x_eta > 0)
    h1 = np.hypot(m.X[1] - m.X[0], m.Y[1] - m.Y[0])
    assert np.max(np.abs(h1 - 0.5)) < 1e-3
    far = np.hypot(m.X[-1], m.Y[-1])
    assert 0.95 * 240.0 < far.min() and far.max() < 1.05 * 240.0


def test_topology_cut_segments_and_mirror():
    m = small_mesh()
    g = Grid.from_mesh(m)
    nA, s, nB, ni = 48, 30, 48, m.ni
    assert g.segments == [(0, nA + 1, True), (nA + s, nB + 1, True)]
    cut = np.flatnonzero(g.cut_col)
    assert np.array_equal(cut, np.r_[nA + 1:nA + s, nA + s + nB + 1:ni])
    assert np.array_equal(np.flatnonzero(g.wall_col), np.r_[0:nA + 1, nA + s:nA + s + nB + 1])
    # the mirror map is an involution that swaps the junction copies
    cols = np.arange(ni)
    assert np.array_equal(g.mirror(g.mirror(cols)), cols)
    assert g.mirror(0) == nA and g.mirror(nA + s) == nA + s + nB
    # node (i, -1) of a cut column is the node below the slit: the mirror
    # image of (i, 1) in the axis
    for i in cut:
        x, y = g.neighbour_pos(m.X, m.Y, 0, -1)
        assert x[0, i] == m.X[1, i] and y[0, i] == -m.Y[1, i]
    # far field: the outer row only; stencils shift up on the wall columns only
    far = boundary_nodes(g)
    assert far.sum() == ni and np.all(far[-1])
    ic, jc = stencil_centres(g)
    assert np.array_equal(jc[0] == 1, g.wall_col) and np.all(ic == g.ii)


def test_uniform_pressure_gives_zero_force_on_each_body():
    m = small_mesh()
    g = Grid.from_mesh(m)
    shape = m.X.shape
    f, gg = L.equilibrium_populations(np.full(shape, 1.2), np.zeros(shape), np.zeros(shape),
                                      np.full(shape, 0.3), 1.4)
    scale = 1.2 * 0.3 * np.pi * 30.0
    for k, ea in ((0, (-45.0, 0.0)), (1, (45.0, 0.0))):
        Fx, Fy, M = FO.wall_force(g, f, gg, m.X, m.Y, 1.4, 0.01, 0.71, 0.1, ea, seg=k)
        assert abs(Fx) < 1e-13 * scale and abs(Fy) < 1e-13 * scale
        assert abs(M) < 1e-11 * scale * 30.0
    # the polygons are the two circles, each node once
    assert len(FO.wall_polygon(g, 0)) == 48 and len(FO.wall_polygon(g, 1)) == 48


def test_regions_of_influence_move_their_own_nodes():
    c = synth.small_tandem_case()
    X, Y = c.mesh.X, c.mesh.Y
    b0, b1 = c.bodies
    states = [(1.5, 0.1, 0, 0), (-0.7, -0.2, 0, 0)]
    b0 = replace(b0, dof=0)
    b1 = replace(b1, dof=0)
    x, y = deformed_positions(X, Y, [b0, b1], states)
    r0, r1 = blend_factors(X, Y, [b0, b1])
    for b, st, r in ((b0, states[0], r0), (b1, states[1], r1)):
        rig = r == 0.0
        gx, gy = rigid_map(X[rig], Y[rig], b, st[0], st[1])
        assert rig.sum() > 100
        assert np.max(np.abs(x[rig] - gx)) < 1e-12 and np.max(np.abs(y[rig] - gy)) < 1e-12
    out = (r0 == 1.0) & (r1 == 1.0)
    assert np.array_equal(x[out], X[out]) and np.array_equal(y[out], Y[out])
    # a linked body moves with its master's rigid map about the master's axis
    bl = replace(b1, link=0)
    x2, y2 = deformed_positions(X, Y, [b0, bl], [states[0], states[0]])
    rig = r1 == 0.0
    gx, gy = rigid_map(X[rig], Y[rig], b0, states[0][0], states[0][1])
    assert np.max(np.abs(x2[rig] - gx)) < 1e-12 and np.max(np.abs(y2[rig] - gy)) < 1e-12
    # overlapping regions are refused
    with pytest.raises(AssertionError):
        blend_factors(X, Y, [b0, replace(b1, r_blend=75.0)])


def test_flow_along_the_axis_stays_mirror_symmetric():
    c = synth.small_tandem_case(h0_frac=0.0)
    bodies = [replace(b, dof=DOF_FIXED) for b in c.bodies]
    ora = OracleSolver(c.mesh, c.fluid, bodies, c.rho, c.ux, c.uy, c.T)
    ora.run(30)
    g = ora.grid
    my = g.mirror(np.arange(c.mesh.ni))
    for F in (ora.f, ora.g):
        for k in range(9):
            assert np.max(np.abs(F[k] - F[REFLECT_Y[k]][:, my])) < 1e-13, k
    rho, ux, uy, _, T = ora.macroscopic()
    assert np.max(np.abs(uy)) > 1e-3 * c.info["U"]
    for hist in ora.histories:
        h = np.array(hist)
        assert np.max(np.abs(h[:, 2])) < 1e-10 * np.max(np.abs(h[:, 1]))
        assert np.max(np.abs(h[:, 3])) < 1e-10 * np.max(np.abs(h[:, 1])) * 30.0


def test_linked_pair_equals_two_half_cylinders_under_symmetry():
    """Gas at rest, both cylinders start 0.02 D above the axis.  The flow is
    mirror-symmetric about the bisector, so both walls carry the same load F.
    The linked pair (m, k; load F_0 + F_1) and two independent cylinders of
    m/2, k/2 (load F each) obey the same equation."""
    c = synth.small_tandem_case(linked=True, h0_frac=0.02)
    fl = replace(c.fluid, u_inf=(0.0, 0.0))
    linked = OracleSolver(c.mesh, fl, c.bodies)
    b0 = c.bodies[0]
    half = replace(b0, m=0.5 * b0.m, k_h=0.5 * b0.k_h)
    indep = OracleSolver(c.mesh, fl, [half, replace(half, center=c.bodies[1].center,
                                                    ea=c.bodies[1].ea)])
    n = 40
    linked.run(n)
    indep.run(n)
    hl = np.array(linked.histories[0])
    hi0 = np.array(indep.histories[0])
    hi1 = np.array(indep.histories[1])
    # the body moved and carried a load
    assert np.max(np.abs(hl[:, 4] - hl[0, 4])) > 1e-5 * 0.6
    assert np.max(np.abs(hl[:, 2])) > 0
    hscale = np.max(np.abs(hl[:, 4]))
    assert np.max(np.abs(hi0[:, 4] - hl[:, 4])) < 1e-10 * hscale
    assert np.max(np.abs(hi1[:, 4] - hl[:, 4])) < 1e-10 * hscale
    # the linked body follows its master and reports its own load
    hl1 = np.array(linked.histories[1])
    assert np.array_equal(hl1[:, 4], hl[:, 4])
    fscale = np.max(np.abs(hl[:, 2]))
    assert np.max(np.abs(hl1[:, 2] - hl[:, 2])) < 1e-9 * fscale      # F_1 = F_0 by symmetry
    # mirror symmetry about the bisector of the populations
    g = linked.grid
    nA, s, nB = 48, 30, 48
    mx = (nA + s + nB - np.arange(c.mesh.ni)) % c.mesh.ni
    for F in (linked.f, linked.g):
        for k in range(9):
            assert np.max(np.abs(F[k] - F[REFLECT_X[k]][:, mx])) < 1e-13, k
    # drag components cancel between the mirror-image walls (to the rounding
    # of a pressure-force sum, whose scale is p times the perimeter)
    assert np.max(np.abs(hl1[:, 1] + hl[:, 1])) < 1e-13 * (1.0 / 3.0) * np.pi * 30.0


def test_linked_pair_integrates_the_summed_load():
    """In a stream (no symmetry) the linked pair's equation m h'' + k h = F_0 + F_1
    is checked step by step against the exact solution for a load frozen over
    the step, h(dt) = h_eq + (h - h_eq) cos(w dt) + (v / w) sin(w dt) with
    h_eq = F / k (RK4's error is O((w dt)^5), far below the tolerance), and the
    downstream load is large enough that dropping it would fail the check."""
    c = synth.small_tandem_case(linked=True, h0_frac=0.02)
    ora = OracleSolver(c.mesh, c.fluid, c.bodies, c.rho, c.ux, c.uy, c.T)
    b = c.bodies[0]
    w = np.sqrt(b.k_h / b.m)
    dt = c.fluid.dt
    worst = 0.0
    sens = 0.0
    for n in range(15):
        h, v = ora.states[0][0], ora.states[0][2]
        ora.step()
        F0, F1 = ora.histories[0][-1][2], ora.histories[1][-1][2]
        heq = (F0 + F1) / b.k_h
        exact = heq + (h - heq) * np.cos(w * dt) + v / w * np.sin(w * dt)
        worst = max(worst, abs(ora.states[0][0] - exact))
        assert ora.states[1][0] == ora.states[0][0]
        alone = F0 / b.k_h + (h - F0 / b.k_h) * np.cos(w * dt) + v / w * np.sin(w * dt)
        sens = max(sens, abs(alone - exact))
    tol = 1e-13 * abs(c.bodies[0].h0)
    assert worst < tol
    # dropping F1 would move the state by far more than the tolerance
    assert sens > 1e3 * tol
