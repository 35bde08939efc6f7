"""Oracle pins for the forced-start-then-release body protocol and for the
distance-field blending (the airfoil workflow of Sec. V and the slender-body
variant of the blending region suggested in Sec. II.D)."""

import math
from dataclasses import replace

import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import body as B
from oracle.mesh import Grid, blend_factor, deformed_positions, distance_to_wall
from oracle.forces import wall_polygon


def pp_body(**kw):
    args = dict(dof=2, m=3.0, S_a=0.4, I_a=1.1, k_h=0.7, k_a=2.3, ea=(0.0, 0.0),
                pitch_amp=math.radians(1.0), pitch_freq=0.2, release_time=4.0)
    args.update(kw)
    return synth.BodyParams(**args)


def test_forced_start_follows_the_prescribed_motion_then_releases():
    b = pp_body()
    dt = 0.05                      # omega dt ~ 0.08: RK4 global error ~1e-5 over 400 steps
    s = B.initial_state(b)
    assert np.array_equal(s, B.prescribed_state(b, 0.0))
    n_rel = int(round(b.release_time / dt))
    for n in range(n_rel):
        s = B.advance(b, s, 123.0, -7.0, (n + 1) * dt, dt)     # loads ignored while forced
        assert np.array_equal(s, B.prescribed_state(b, (n + 1) * dt))
    # free: without loads the section oscillates about its equilibrium, as the
    # exact solution of M y'' + K y = 0 from the release state (RK4 error only)
    Mm = np.array([[b.m, b.S_a], [b.S_a, b.I_a]])
    K = np.diag([b.k_h, b.k_a])
    A = np.zeros((4, 4))
    A[:2, 2:] = np.eye(2)
    A[2:, :2] = -np.linalg.solve(Mm, K)
    y0 = s.copy()
    for k in range(1, 401):
        s = B.advance(b, s, 0.0, 0.0, (n_rel + k) * dt, dt)
    exact = expm(A * 400 * dt) @ y0
    assert np.max(np.abs(s - exact)) <= 1e-4 * np.max(np.abs(y0))
    # and the load acts again once released
    s2 = B.advance(b, y0, 1.0, 0.0, (n_rel + 1) * dt, dt)
    assert not np.allclose(s2, B.advance(b, y0, 0.0, 0.0, (n_rel + 1) * dt, dt))


def test_release_time_zero_is_the_plain_dof():
    b = pp_body(release_time=0.0, a0=0.01)
    s = B.initial_state(b)
    assert np.array_equal(s, [0.0, 0.01, 0.0, 0.0])


def test_distance_to_wall_against_dense_edge_sampling():
    m = synth.cgrid_mesh(16, 64, 32, 40.0, 0.5, 4.0)
    g = Grid.from_mesh(m)
    cols = wall_polygon(g)
    px, py = m.X[0, cols], m.Y[0, cols]
    rng = np.random.default_rng(3)
    pts_x = rng.uniform(-20, 60, size=(4, 50))
    pts_y = rng.uniform(-30, 30, size=(4, 50))
    d = distance_to_wall(pts_x, pts_y, px, py)
    # dense sampling of every edge: an upper bound within half a sample spacing
    t = np.linspace(0.0, 1.0, 2001)
    qx = (px[:, None] + (np.roll(px, -1) - px)[:, None] * t).ravel()
    qy = (py[:, None] + (np.roll(py, -1) - py)[:, None] * t).ravel()
    dd = np.sqrt((pts_x.ravel()[:, None] - qx) ** 2 + (pts_y.ravel()[:, None] - qy) ** 2).min(axis=1)
    seg = np.max(np.hypot(np.diff(px), np.diff(py)))
    assert np.all(d.ravel() <= dd + 1e-12)
    assert np.all(d.ravel() >= dd - 0.5 * seg / 2000 - 1e-12)


def test_distance_blending_on_a_circle_matches_radial_up_to_the_chord_sag():
    c = synth.cylinder_viv_case(n_r=32, n_theta=64, D=20.0, first_cell_frac=0.05,
                                r_far_D=8.0, blend_D=3.0)
    m = c.mesh
    g = Grid.from_mesh(m)
    cols = wall_polygon(g)
    d = distance_to_wall(m.X, m.Y, m.X[0, cols], m.Y[0, cols])
    R = 10.0
    r = np.hypot(m.X, m.Y)
    sag = R * (1.0 - math.cos(math.pi / m.ni))
    assert np.all(d <= r - R + sag + 1e-9) and np.all(d >= r - R - 1e-9)


def test_distance_blending_keeps_the_wall_rigid():
    c = synth.small_airfoil_case()
    m = c.mesh
    body = replace(c.bodies[0], blend_mode=1, r_rigid=1.0, r_blend=60.0)
    g = Grid.from_mesh(m)
    cols = wall_polygon(g)
    wall = (m.X[0, cols], m.Y[0, cols])
    r = blend_factor(m.X, m.Y, body, wall)
    assert np.all(r[0, m.n_wake:m.ni - m.n_wake] == 0.0)
    state = [np.array([0.3, 0.05, 0.0, 0.0])]
    x, y = deformed_positions(m.X, m.Y, [body], state, wall)
    # rigid motion of the wall: translation 0.3 along y, rotation 0.05 about the EA
    ex, ey = body.ea
    ca, sa = math.cos(0.05), math.sin(0.05)
    X0, Y0 = m.X[0], m.Y[0]
    gx = ex + ca * (X0 - ex) - sa * (Y0 - ey)
    gy = ey + 0.3 + sa * (X0 - ex) + ca * (Y0 - ey)
    w = slice(m.n_wake, m.ni - m.n_wake)
    assert np.max(np.abs(x[0, w] - gx[w])) < 1e-12 and np.max(np.abs(y[0, w] - gy[w])) < 1e-12
    # far nodes stay put
    far = r == 1.0
    assert np.any(far) and np.array_equal(x[far], m.X[far])
