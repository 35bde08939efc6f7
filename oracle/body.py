"""Rigid-body structural models in float64 (paper Sec. IV).  Test
infrastructure only.

State s = (h, alpha, hdot, alphadot): plunge h along +y, pitch alpha
counter-clockwise about the elastic axis.

1DOF (Sec. IV.A):  m h'' + k_h h = F_y                (undamped)
2DOF (Sec. IV.B):  m h'' + S_a a'' + k_h h = F_y
                   S_a h'' + I_a a'' + k_a a = M_EA
integrated with the classical fourth-order Runge-Kutta method over one time
step with the fluid load frozen (staggered weak coupling, Sec. III), or, in
the sub-iterations of strong coupling, varying linearly over the step.
Prescribed motion: h(t) = A_h sin(2 pi f_h t), alpha(t) = A_a sin(2 pi f_a t).
A fixed body keeps its initial state.

Forced start then release (Sec. V, the airfoil's protocol: a forced pitching
perturbation for a number of periods, after which the section moves freely):
a 1DOF or 2DOF body with release_time > 0 follows the prescribed motion while
t^{n+1} <= release_time and integrates its ODE from the state reached
afterwards.  Reading: the plunge is held by the forcing unless a heave
amplitude is given; the first free step starts from the prescribed state of
the last forced level.
"""

from __future__ import annotations

import math

import numpy as np

DOF_PRESCRIBED = 0
DOF_HEAVE = 1
DOF_PITCH_PLUNGE = 2
DOF_FIXED = 3


def accelerations(body, h, a, Fy, M):
    """Solve the mass-matrix system for (h'', a'')."""
    if body.dof == DOF_HEAVE:
        return (Fy - body.k_h * h) / body.m, 0.0
    if body.dof == DOF_PITCH_PLUNGE:
        r1 = Fy - body.k_h * h
        r2 = M - body.k_a * a
        Mm = np.array([[body.m, body.S_a], [body.S_a, body.I_a]])
        hdd, add = np.linalg.solve(Mm, np.array([r1, r2]))
        return float(hdd), float(add)
    raise ValueError("no dynamics for this dof")


def rk4_step(body, state, Fy, M, dt, Fy1=None, M1=None):
    """One RK4 step of the first-order system y' = (hdot, adot, h'', a'').

    The load is (Fy, M) throughout, or, with (Fy1, M1), varies linearly in
    time from (Fy, M) at the start of the step to (Fy1, M1) at its end (each
    stage takes the load at its own time)."""
    if Fy1 is None:
        Fy1, M1 = Fy, M

    def rhs(y, c):
        hdd, add = accelerations(body, y[0], y[1], Fy + c * (Fy1 - Fy), M + c * (M1 - M))
        return np.array([y[2], y[3], hdd, add])

    y = np.asarray(state, dtype=np.float64)
    k1 = rhs(y, 0.0)
    k2 = rhs(y + 0.5 * dt * k1, 0.5)
    k3 = rhs(y + 0.5 * dt * k2, 0.5)
    k4 = rhs(y + dt * k3, 1.0)
    return y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def prescribed_state(body, t):
    wh = 2.0 * math.pi * body.heave_freq
    wa = 2.0 * math.pi * body.pitch_freq
    return np.array([body.heave_amp * math.sin(wh * t),
                     body.pitch_amp * math.sin(wa * t),
                     body.heave_amp * wh * math.cos(wh * t),
                     body.pitch_amp * wa * math.cos(wa * t)])


def forced(body, t):
    """True while a released body still follows its prescribed start."""
    rt = getattr(body, "release_time", 0.0)
    return body.dof in (DOF_HEAVE, DOF_PITCH_PLUNGE) and rt > 0.0 and t <= rt


def initial_state(body):
    if body.dof == DOF_PRESCRIBED or forced(body, 0.0):
        return prescribed_state(body, 0.0)
    return np.array([body.h0, body.a0, body.hd0, body.ad0], dtype=np.float64)


def advance(body, state, Fy, M, t_next, dt, Fy1=None, M1=None):
    """State at t^{n+1} from the state at t^n and the frozen load at t^n, or
    (with Fy1, M1) the load varying linearly to (Fy1, M1) at t^{n+1}."""
    if body.dof == DOF_PRESCRIBED or forced(body, t_next):
        return prescribed_state(body, t_next)
    if body.dof == DOF_FIXED:
        return np.asarray(state, dtype=np.float64).copy()
    return rk4_step(body, state, Fy, M, dt, Fy1, M1)
