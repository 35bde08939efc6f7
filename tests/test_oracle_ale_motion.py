"""P19: mesh-motion consistency of the whole ALE step (Sec. II.A transformed
velocity, Sec. II.B semi-Lagrangian propagation of every population).

A pressure pulse is run on a periodic mesh twice: once on the static mesh and
once on a mesh that moves and, after one full period of a prescribed motion,
is back where it started.  The two runs solve the same physical problem, so
their densities at the nodes must agree up to the interpolation and
departure-point errors of the scheme, and that difference must fall under
refinement (the pulse width, the motion amplitude and the period scaled with
the mesh).  The planted mistake is the rest populations kept at their node
(c^_0 = -g^{-1} V_G taken as zero): it leaves an error of the pulse's own
order that does not fall with refinement.
"""

import math

import numpy as np
import pytest

import synth
import oracle.stream as S
from oracle.solver import OracleSolver

AMP = 1e-3


def pulse_case(n, kind):
    mesh = synth.periodic_sine_mesh(n, 0.05 * n / 64)
    dt = 1.0 / 3.0
    fluid = synth.FluidParams(gamma=1.4, Pr=0.71, mu=0.01, rho_inf=1.0, T_inf=1.0 / 3.0,
                              u_inf=(0.0, 0.0), dt=dt)
    steps = n
    period = steps * dt
    c = 0.5 * n
    if kind == "translate":
        # every node in the rigid zone: the whole box moves along y and back
        body = synth.BodyParams(dof=0, center=(c, c), ea=(c, c), r_rigid=10.0 * n,
                                r_blend=20.0 * n, heave_amp=2.0 * n / 32,
                                heave_freq=1.0 / period)
        pc = (c, c)
    else:
        # a disk turning by up to 0.5 rad and back, blended into the static box;
        # the pulse sits off the axis so the turning mesh crosses its gradient
        body = synth.BodyParams(dof=0, center=(c, c), ea=(c, c), r_rigid=0.1 * n,
                                r_blend=0.4 * n, pitch_amp=0.5, pitch_freq=1.0 / period)
        pc = (c + n / 8, c)
    sig = n / 16
    r2 = (mesh.X - pc[0]) ** 2 + (mesh.Y - pc[1]) ** 2
    rho = 1.0 + AMP * np.exp(-r2 / (2.0 * sig ** 2))
    zero = np.zeros_like(mesh.X)
    T = np.full_like(mesh.X, 1.0 / 3.0)
    return mesh, fluid, body, steps, (rho, zero, zero.copy(), T)


def run(mesh, fluid, bodies, steps, fields, keep_rest=False):
    s = OracleSolver(mesh, fluid, bodies, *fields)
    orig = S.transformed_velocities
    if keep_rest:
        def planted(*a, **k):
            out = orig(*a, **k)
            out[0] = (np.zeros_like(out[0][0]), np.zeros_like(out[0][1]))
            return out
        S.transformed_velocities = planted
    try:
        s.run(steps)
    finally:
        S.transformed_velocities = orig
    if bodies:
        # the motion is periodic: the mesh is back at its start
        x, y = s.positions(s.states)
        assert np.max(np.abs(x - mesh.X)) < 1e-9 and np.max(np.abs(y - mesh.Y)) < 1e-9
    return s.macroscopic()[0]


def errors(kind, n):
    mesh, fluid, body, steps, fields = pulse_case(n, kind)
    r_static = run(mesh, fluid, [], steps, fields)
    r_moving = run(mesh, fluid, [body], steps, fields)
    r_planted = run(mesh, fluid, [body], steps, fields, keep_rest=True)
    e = np.max(np.abs(r_moving - r_static)) / AMP
    ep = np.max(np.abs(r_planted - r_static)) / AMP
    return e, ep


@pytest.mark.parametrize("kind,min_order,max_err64", [("translate", 1.3, 0.01),
                                                      ("rotate", 0.6, 0.05)])
def test_pulse_on_moving_mesh_matches_static_run(kind, min_order, max_err64):
    """Translation: the whole periodic box moves by up to 4 cells (n = 64) and
    back; rotation: a blended disk turns by up to 0.5 rad and back.  The
    departure point X - dt c^ is first order in time when c^ varies over the
    step, so the error falls at least at first order; the translation also
    sees the spatial order of the interpolation."""
    e32, p32 = errors(kind, 32)
    e64, p64 = errors(kind, 64)
    order = math.log2(e32 / e64)
    assert order >= min_order, (e32, e64)
    assert e64 <= max_err64
    # the rest populations kept at their node: an error of the pulse's order
    # that refinement does not reduce
    assert p64 > 4.0 * e64 and p64 > 0.15, (p32, p64)
    assert p64 >= 0.9 * p32


def test_rest_population_departure_on_translating_mesh():
    """On a rigidly translating mesh g = I: the rest populations' departure
    point is X + dt V_G, and a static mesh keeps them at their node bitwise."""
    mesh, fluid, body, steps, fields = pulse_case(32, "translate")
    s = OracleSolver(mesh, fluid, [body], *fields)
    x0, y0 = s.positions(s.states)
    st1 = [np.asarray(S_) for S_ in s._advance_bodies([(0.0, 0.0, 0.0)])]
    x1, y1 = s.positions(st1)
    dt = fluid.dt
    VGx, VGy = (x1 - x0) / dt, (y1 - y0) / dt
    assert np.max(np.abs(VGy)) > 0.05
    chat = S.transformed_velocities(s.grid, s.X, s.Y, x1, y1, VGx, VGy)
    a, b, miss = S.departure_offsets(s.grid, s.X, s.Y, chat[0][0], chat[0][1], dt)
    # interior of a unit-spaced mesh in x: index offsets equal the physical
    # offset dt V_G to the accuracy of the mesh's small sine deformation
    assert np.allclose(b, dt * VGy, atol=0.05 * dt * np.max(np.abs(VGy)))
    assert np.max(np.abs(a)) < 0.05 * dt * np.max(np.abs(VGy))
    zero = np.zeros_like(s.X)
    chat0 = S.transformed_velocities(s.grid, s.X, s.Y, s.X, s.Y, zero, zero)
    a0, b0, _ = S.departure_offsets(s.grid, s.X, s.Y, chat0[0][0], chat0[0][1], dt)
    assert np.all(a0 == 0.0) and np.all(b0 == 0.0)
