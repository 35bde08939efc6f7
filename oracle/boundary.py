"""Boundary conditions in float64 (paper Sec. III.A).  Test infrastructure only.

Wall (row j = 0 of an O-grid): populations whose departure point lies inside
the body are replaced with Grad's approximation built from target values
(Sec. III.A.1):

    f_i = f_i^eq(rho_t, u_t, T_t) + dt f_i^(1),   g_i = g_i^eq(...) + dt g_i^(1)

Readings taken where the text is silent or garbled:
* u_t is the wall-node mesh velocity V_G (no slip on a moving wall; zero for a
  body at rest, as printed).
* rho_t, T_t are the values at B, the point at distance dt along the unit wall
  normal (zero normal gradient).  The wall lies in the rigid region of the
  blended mesh, so B is placed in the undeformed frame and located with the
  bilinear cell map.  B is interpolated with the 9-node element centred on
  the node of row 1; the wall-row values in that element are those of the
  previous time step (the current ones are being constructed).
* P^(1) = -(1/omega) rho T [S - (1/C_v)(div u) I] (the printed
  "(S - 1/C_v)(div u) I" has a misplaced parenthesis; this form is the
  Navier-Stokes-Fourier stress of Sec. II.C).
* f^(1) = W_i P^(1):(c c - T I)/(2 T^2).
* gradients are FE derivatives on the mesh at t^{n+1}: centred along the wall,
  one-sided into the fluid, with the wall row holding the target values.

Far field (row j = nj - 1): all populations are set to equilibrium
(Sec. III.A.2).  Reading: a node is an inlet when u_inf . n_out < 0, with
n_out the outward normal of the far-field row; inlets take the free-stream
values, outlets copy rho, u, T from the adjacent interior node (zero gradient).
"""

from __future__ import annotations

import numpy as np

from . import lattice as L
from .stream import bilinear_inverse, lagrange_1d


def wall_normals_undeformed(grid, X, Y):
    """Unit normal of the wall row pointing into the fluid, from the centred
    tangent t = X_{i+1} - X_{i-1}: n = rot_{+90}(t)/|t| (meshes have
    det(dX/dxi) > 0 with j pointing into the fluid)."""
    xp, yp = grid.neighbour_pos(X, Y, 1, 0)
    xm, ym = grid.neighbour_pos(X, Y, -1, 0)
    tx = (xp - xm)[0]
    ty = (yp - ym)[0]
    n = np.hypot(tx, ty)
    return -ty / n, tx / n


def interpolate_B(grid, X, Y, field_row0, field_rows12, dt):
    """Value at B = X_A + dt n (undeformed frame) for every wall node.

    field_row0: wall-row values [ni]; field_rows12: full field [nj, ni] whose
    rows 1 and 2 are used.
    """
    nx, ny = wall_normals_undeformed(grid, X, Y)
    ni = grid.ni
    Bx = dt * nx
    By = dt * ny                      # B - X_A
    a = np.full(ni, np.nan)
    b = np.full(ni, np.nan)
    found = np.zeros(ni, dtype=bool)
    for di0 in (-1, 0):
        corners = []
        for (ci, cj) in ((0, 0), (1, 0), (0, 1), (1, 1)):
            px, py = grid.neighbour_pos(X, Y, di0 + ci, cj)
            corners.append((px[0] - X[0], py[0] - Y[0]))
        s, t, _ = bilinear_inverse(*corners, Bx, By)
        ok = (s >= -1e-12) & (s <= 1 + 1e-12) & (t >= -1e-12) & (t <= 1 + 1e-12)
        take = ok & ~found
        a = np.where(take, di0 + s, a)
        b = np.where(take, t, b)
        found |= take
    if not np.all(found):
        raise ValueError("point B outside the first cell row (dt larger than the wall cell)")
    # element centred on (i, 1): rows 0, 1, 2
    vals = np.stack([field_row0, field_rows12[1], field_rows12[2]])
    bc = b - 1.0
    out = np.zeros(ni)
    ii = np.arange(ni)
    for p in (-1, 0, 1):
        La = lagrange_1d(p, a)
        for q in (-1, 0, 1):
            Lb = lagrange_1d(q, bc)
            out = out + La * Lb * vals[q + 1, (ii + p) % ni]
    return out


def wall_grad_bc(grid, X, Y, x1, y1, VGx, VGy, f_new, g_new, missing,
                 f_old, g_old, gamma, mu, Pr, dt):
    """Fill the missing wall populations of (f_new, g_new) in place with
    Grad's approximation (Sec. III.A.1).  Returns the targets (rho, ux, uy, T)."""
    Cv, Cp = L.specific_heats(gamma)
    # macroscopic fields of the freshly streamed populations (rows >= 1 complete)
    f_fill = np.where(np.isnan(f_new), 0.0, f_new)
    g_fill = np.where(np.isnan(g_new), 0.0, g_new)
    with np.errstate(invalid="ignore", divide="ignore"):
        rho, ux, uy, E, T = L.macroscopic(f_fill, g_fill, gamma)
    # previous-step wall values
    rho0, _, _, _, T0 = L.macroscopic(f_old[:, 0, :], g_old[:, 0, :], gamma)

    rho_t = interpolate_B(grid, X, Y, rho0, rho, dt)
    T_t = interpolate_B(grid, X, Y, T0, T, dt)
    ux_t = VGx[0].copy()
    uy_t = VGy[0].copy()
    E_t = Cv * T_t + 0.5 * (ux_t ** 2 + uy_t ** 2)

    # fields with the wall row set to the targets, for the FE gradients
    def with_row0(F, row0):
        G = F.copy()
        G[0] = row0
        return G

    Ux = with_row0(ux, ux_t)
    Uy = with_row0(uy, uy_t)
    TT = with_row0(T, T_t)
    EE = with_row0(E, E_t)
    dux_dx, dux_dy = (v[0] for v in grid.grad(Ux, x1, y1))
    duy_dx, duy_dy = (v[0] for v in grid.grad(Uy, x1, y1))
    dT_dx, dT_dy = (v[0] for v in grid.grad(TT, x1, y1))
    dE_dx, dE_dy = (v[0] for v in grid.grad(EE, x1, y1))

    omega, omega1 = L.relaxation_rates(rho_t, T_t, mu, Pr, dt)
    # strain rate S = grad u + grad u^T, (grad u)_ab = d_a u_b
    Sxx = 2.0 * dux_dx
    Syy = 2.0 * duy_dy
    Sxy = dux_dy + duy_dx
    div = dux_dx + duy_dy
    pref = -(1.0 / omega) * rho_t * T_t
    P1xx = pref * (Sxx - div / Cv)
    P1yy = pref * (Syy - div / Cv)
    P1xy = pref * Sxy
    # q^(1) = -(2/omega1) rho C_p T grad T + 2 u . P^(1)
    q1x = -(2.0 / omega1) * rho_t * Cp * T_t * dT_dx + 2.0 * (ux_t * P1xx + uy_t * P1xy)
    q1y = -(2.0 / omega1) * rho_t * Cp * T_t * dT_dy + 2.0 * (ux_t * P1xy + uy_t * P1yy)
    # R^(1) = -(2/omega1) rho T [S (E + 2T) + u (grad E)^T + grad E u^T]
    rpref = -(2.0 / omega1) * rho_t * T_t
    R1xx = rpref * (Sxx * (E_t + 2.0 * T_t) + 2.0 * ux_t * dE_dx)
    R1yy = rpref * (Syy * (E_t + 2.0 * T_t) + 2.0 * uy_t * dE_dy)
    R1xy = rpref * (Sxy * (E_t + 2.0 * T_t) + ux_t * dE_dy + uy_t * dE_dx)

    fe = L.feq(rho_t, ux_t, uy_t, T_t)
    ge = L.geq(rho_t, ux_t, uy_t, E_t, T_t)
    W = L.weights(T_t)
    for i in range(L.Q):
        cx, cy = L.CX[i], L.CY[i]
        f1 = W[i] * (P1xx * (cx * cx - T_t) + 2.0 * P1xy * cx * cy
                     + P1yy * (cy * cy - T_t)) / (2.0 * T_t * T_t)
        g1 = W[i] * ((q1x * cx + q1y * cy) / T_t
                     + (R1xx * (cx * cx - T_t) + 2.0 * R1xy * cx * cy
                        + R1yy * (cy * cy - T_t)) / (2.0 * T_t * T_t))
        m = missing[i, 0]
        f_new[i, 0] = np.where(m, fe[i] + dt * f1, f_new[i, 0])
        g_new[i, 0] = np.where(m, ge[i] + dt * g1, g_new[i, 0])
    return rho_t, ux_t, uy_t, T_t


def farfield_outward_normal(grid, X, Y):
    """Outward normal (not normalised) of the far-field row: rot_{+90} of the
    centred tangent, which points toward increasing j."""
    xp, yp = grid.neighbour_pos(X, Y, 1, 0)
    xm, ym = grid.neighbour_pos(X, Y, -1, 0)
    tx = (xp - xm)[-1]
    ty = (yp - ym)[-1]
    return -ty, tx


def farfield_bc(grid, X, Y, f_new, g_new, gamma, rho_inf, u_inf, T_inf):
    """Equilibrium populations on the far-field row (Sec. III.A.2)."""
    nx, ny = farfield_outward_normal(grid, X, Y)
    inflow = (u_inf[0] * nx + u_inf[1] * ny) < 0.0
    rho_in, ux_in, uy_in, _, T_in = L.macroscopic(f_new[:, -2, :], g_new[:, -2, :], gamma)
    rho = np.where(inflow, rho_inf, rho_in)
    ux = np.where(inflow, u_inf[0], ux_in)
    uy = np.where(inflow, u_inf[1], uy_in)
    T = np.where(inflow, T_inf, T_in)
    fe, ge = L.equilibrium_populations(rho, ux, uy, T, gamma)
    f_new[:, -1, :] = fe
    g_new[:, -1, :] = ge
    return inflow
