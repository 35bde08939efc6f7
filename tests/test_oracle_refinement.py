"""P17: drag of a fixed cylinder under mesh refinement (paper Sec. III force
on the Sec. II mesh; the paper prints no drag values for this case, so the
absolute value is not pinned, only its convergence).

A fixed cylinder at Re 20, Ma 0.2, on three O-grids refined by two in both
directions (16 x 8, 32 x 16, 64 x 32 nodes; square wall cells of pi D / n;
far field at 8 D; D = n / 4 lattice units), from the same start in units of
D (potential flow with a boundary layer of width D / 2), stepped to the same
time 1 D / U.  The drag coefficient averaged over the second half of that
time converges: the differences between successive levels fall with an
observed order between 1.5 and 3.5 (second order expected of the scheme's
quadratic elements and centred derivatives).  The mesh and the start are
mirror-symmetric about the flow direction, and on the finest mesh the lift
stays at round-off.
"""

import math

import numpy as np

import synth
from synth.configs import DOF_FIXED
from oracle.solver import OracleSolver

RE, MA, FAR_D = 20.0, 0.2, 8.0


def drag_coefficient(n_theta):
    D = n_theta / 4.0
    first = math.pi * D / n_theta
    mesh = synth.ogrid_mesh(n_theta // 2, n_theta, D, first, FAR_D * D)
    U = MA * synth.configs.sound_speed(1.4, 1.0 / 3.0)
    dt = first / 3.0
    fluid = synth.FluidParams(gamma=1.4, Pr=0.71, mu=U * D / RE, rho_inf=1.0, T_inf=1.0 / 3.0,
                              u_inf=(U, 0.0), dt=dt)
    body = synth.BodyParams(dof=DOF_FIXED, center=(0.0, 0.0), ea=(0.0, 0.0),
                            r_rigid=0.5 * D, r_blend=2.0 * D)
    r, ux, uy, T = synth.configs.cylinder_start_fields(mesh, D, U, 1.0, 1.0 / 3.0, 0.5 * D)
    ora = OracleSolver(mesh, fluid, [body], r, ux, uy, T)
    n = int(round(D / U / dt))
    ora.run(n)
    h = np.array(ora.history)
    q = 0.5 * U * U * D
    cd = float(np.mean(h[n // 2:, 1]) / q)
    cl = float(np.max(np.abs(h[:, 2])) / q)
    return cd, cl


def test_cylinder_drag_converges_under_refinement():
    (c1, _), (c2, _), (c3, l3) = (drag_coefficient(n) for n in (16, 32, 64))
    assert all(np.isfinite(c) and c > 0 for c in (c1, c2, c3))
    order = math.log2(abs(c2 - c1) / abs(c3 - c2))
    print(f"C_D = {c1:.4f}, {c2:.4f}, {c3:.4f}; observed order {order:.2f}")
    assert 1.5 <= order <= 3.5, (c1, c2, c3, order)
    assert l3 <= 1e-12
