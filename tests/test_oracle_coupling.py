"""Oracle pins for strong coupling by sub-iterations: one sub-iteration is the
staggered scheme, the sub-iterations contract, the accepted structure state
solves the body equation exactly for the load that varies linearly from F^n
to the load of the accepted fluid state (closed-form solution of
m h'' + k h = F0 + (F1 - F0) t / dt), relaxation changes the path, not the
limit, and a fixed body is untouched."""

from dataclasses import replace

import numpy as np

import synth
from oracle.solver import OracleSolver

DOF_FIXED = 3


def light_cylinder(mstar=0.5):
    return synth.cylinder_viv_case(n_r=32, n_theta=64, D=20.0, first_cell_frac=0.05,
                                   r_far_D=8.0, blend_D=3.0, h0_frac=0.05, mstar=mstar,
                                   ustar=4.0, Ma=0.2, Re=50.0)


def solver(c, K=1, w=1.0, bodies=None):
    o = OracleSolver(c.mesh, c.fluid, bodies if bodies is not None else c.bodies,
                     c.rho, c.ux, c.uy, c.T)
    o.coupling(K, w)
    return o


def test_one_subiteration_is_the_staggered_scheme():
    c = light_cylinder()
    a, b = solver(c), OracleSolver(c.mesh, c.fluid, c.bodies, c.rho, c.ux, c.uy, c.T)
    a.run(5)
    b.run(5)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.g, b.g)
    assert np.array_equal(np.array(a.history), np.array(b.history))


def test_subiterations_converge_to_the_linear_load_solution():
    c = light_cylinder()
    o = solver(c, K=8)
    body = c.bodies[0]
    w = np.sqrt(body.k_h / body.m)
    dt = c.fluid.dt
    worst = 0.0
    for n in range(10):
        h0, v0 = o.states[0][0], o.states[0][2]
        o.step()
        r = o.residuals
        assert len(r) == 8
        # the change per sub-iteration contracts
        assert r[-1] < 1e-3 * r[0] or r[-1] < 1e-15
        F0 = o.histories[0][-1][2]
        F1 = o.body_forces()[0][1]                # load of the accepted state
        Fd = (F1 - F0) / dt
        exact = (F1 / body.k_h + (h0 - F0 / body.k_h) * np.cos(w * dt)
                 + (v0 - Fd / body.k_h) / w * np.sin(w * dt))
        worst = max(worst, abs(o.states[0][0] - exact) - r[-1])
    assert worst < 1e-13 * abs(c.bodies[0].h0)
    # the load responds to the motion: the converged state differs from the
    # staggered one by far more than the tolerance
    s = solver(c)
    s.run(10)
    assert abs(s.states[0][0] - o.states[0][0]) > 1e3 * 1e-13 * abs(c.bodies[0].h0)


def test_relaxation_changes_the_path_not_the_limit():
    c = light_cylinder()
    a, b = solver(c, K=10, w=1.0), solver(c, K=24, w=0.6)
    a.run(4)
    b.run(4)
    assert b.residuals[-1] < 1e-12 * abs(c.bodies[0].h0)
    hs = abs(c.bodies[0].h0)
    assert abs(a.states[0][0] - b.states[0][0]) < 1e-11 * hs
    assert np.max(np.abs(a.f - b.f)) < 1e-12


def test_subiterations_leave_a_fixed_body_alone():
    c = light_cylinder()
    fixed = [replace(c.bodies[0], dof=DOF_FIXED)]
    a, b = solver(c, K=3, bodies=fixed), solver(c, K=1, bodies=fixed)
    a.run(3)
    b.run(3)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.g, b.g)
    assert all(r == 0.0 for r in a.residuals)
