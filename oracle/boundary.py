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

Far field (row j = nj - 1, and the exit columns of a C-grid): all populations
are set to equilibrium (Sec. III.A.2).  Reading: a node is an inlet when
u_inf . n_out < 0, with n_out the outward normal of its boundary; inlets take
the free-stream values, outlets copy rho, u, T from the adjacent interior node
(zero gradient).

C-grid: the wall is row 0 between the two trailing-edge copies (both are wall
nodes); the cut nodes of row 0 are interior nodes and keep their streamed
values, also where a wall node's tangential derivative reaches them.
"""

from __future__ import annotations

import numpy as np

from . import lattice as L
from .stream import bilinear_inverse, lagrange_1d


def wall_normals_undeformed(grid, X, Y):
    """Unit normal of the wall row pointing into the fluid, from the centred
    tangent t = X_{i+1} - X_{i-1} of index neighbours: n = rot_{+90}(t)/|t|
    (meshes have det(dX/dxi) > 0 with j pointing into the fluid).  Returned
    for every column; only wall columns use it."""
    xp, yp = grid.neighbour_pos(X, Y, 1, 0)
    xm, ym = grid.neighbour_pos(X, Y, -1, 0)
    tx = (xp - xm)[0]
    ty = (yp - ym)[0]
    n = np.hypot(tx, ty)
    with np.errstate(invalid="ignore"):
        return -ty / n, tx / n


def interpolate_B(grid, X, Y, field_row0, field_rows12, dt):
    """Value at B = X_A + dt n (undeformed frame) for every wall node (NaN in
    the other columns).

    field_row0: row-0 values [ni]; field_rows12: full field [nj, ni] whose
    rows 1 and 2 are used.
    """
    nx, ny = wall_normals_undeformed(grid, X, Y)
    ni = grid.ni
    cols = np.flatnonzero(grid.wall_col)
    Bx = dt * nx[cols]
    By = dt * ny[cols]                # B - X_A
    a = np.full(cols.size, np.nan)
    b = np.full(cols.size, np.nan)
    found = np.zeros(cols.size, dtype=bool)
    for di0 in (-1, 0):
        corners = []
        for (ci, cj) in ((0, 0), (1, 0), (0, 1), (1, 1)):
            px, py = grid.neighbour_pos(X, Y, di0 + ci, cj)
            corners.append((px[0, cols] - X[0, cols], py[0, cols] - Y[0, cols]))
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
    out = np.full(ni, np.nan)
    acc = np.zeros(cols.size)
    for p in (-1, 0, 1):
        La = lagrange_1d(p, a)
        si, _, _ = grid.node_index(cols + p, np.zeros_like(cols))
        for q in (-1, 0, 1):
            Lb = lagrange_1d(q, bc)
            acc = acc + La * Lb * vals[q + 1, si]
    out[cols] = acc
    return out


def grad_populations(rho_t, ux_t, uy_t, T_t, E_t, du_x, du_y, dT, dE, gamma, mu, Pr, dt):
    """Grad's approximation f_i = f_i^eq + dt f_i^(1), g_i = g_i^eq + dt g_i^(1)
    (Sec. III.A.1) of all nine populations from the target values and the
    gradients (d/dx, d/dy) of u_x, u_y, T and E at the wall nodes."""
    Cv, Cp = L.specific_heats(gamma)
    dux_dx, dux_dy = du_x
    duy_dx, duy_dy = du_y
    dT_dx, dT_dy = dT
    dE_dx, dE_dy = dE
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
    fw = np.empty((L.Q,) + np.shape(rho_t))
    gw = np.empty_like(fw)
    for i in range(L.Q):
        cx, cy = L.CX[i], L.CY[i]
        f1 = W[i] * (P1xx * (cx * cx - T_t) + 2.0 * P1xy * cx * cy
                     + P1yy * (cy * cy - T_t)) / (2.0 * T_t * T_t)
        g1 = W[i] * ((q1x * cx + q1y * cy) / T_t
                     + (R1xx * (cx * cx - T_t) + 2.0 * R1xy * cx * cy
                        + R1yy * (cy * cy - T_t)) / (2.0 * T_t * T_t))
        fw[i] = fe[i] + dt * f1
        gw[i] = ge[i] + dt * g1
    return fw, gw


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

    # fields with the wall nodes set to the targets, for the FE gradients
    # (cut nodes of a C-grid keep their streamed values)
    wc = grid.wall_col

    def with_row0(F, row0):
        G = F.copy()
        G[0] = np.where(wc, row0, F[0])
        return G

    Ux = with_row0(ux, ux_t)
    Uy = with_row0(uy, uy_t)
    TT = with_row0(T, T_t)
    EE = with_row0(E, E_t)
    dux_dx, dux_dy = (v[0] for v in grid.grad(Ux, x1, y1))
    duy_dx, duy_dy = (v[0] for v in grid.grad(Uy, x1, y1))
    dT_dx, dT_dy = (v[0] for v in grid.grad(TT, x1, y1))
    dE_dx, dE_dy = (v[0] for v in grid.grad(EE, x1, y1))

    fw, gw = grad_populations(rho_t, ux_t, uy_t, T_t, E_t, (dux_dx, dux_dy), (duy_dx, duy_dy),
                              (dT_dx, dT_dy), (dE_dx, dE_dy), gamma, mu, Pr, dt)
    for i in range(L.Q):
        m = missing[i, 0] & wc
        f_new[i, 0] = np.where(m, fw[i], f_new[i, 0])
        g_new[i, 0] = np.where(m, gw[i], g_new[i, 0])
    return rho_t, ux_t, uy_t, T_t


def farfield_nodes(grid, X, Y):
    """Far-field nodes with their outward normals (not normalised) and the
    interior node an outlet copies from (Sec. III.A.2).

    Row nj - 1: n_out = rot_{+90}(dX/di), interior node (i, nj - 2) (its column
    moved off a C-grid exit column).  C-grid exit columns i = 0 and ni - 1
    (rows below nj - 1): n_out = rot_{+90}(dX/dj) at i = 0 and its opposite at
    i = ni - 1, interior nodes (1, j) and (ni - 2, j).  Derivatives are the
    index-space FE derivatives of the undeformed coordinates.
    Returns (jj, ii, nx, ny, jref, iref) as flat arrays.
    """
    X_i, Y_i = grid.d_i(X), grid.d_i(Y)
    X_j, Y_j = grid.d_j(X), grid.d_j(Y)
    ni, nj = grid.ni, grid.nj
    ii = list(range(ni))
    jj = [nj - 1] * ni
    nx = list(-Y_i[nj - 1])
    ny = list(X_i[nj - 1])
    iref = [min(max(i, 1), ni - 2) if grid.cgrid else i for i in range(ni)]
    jref = [nj - 2] * ni
    if grid.cgrid:
        for j in range(nj - 1):
            ii += [0, ni - 1]
            jj += [j, j]
            nx += [-Y_j[j, 0], Y_j[j, ni - 1]]
            ny += [X_j[j, 0], -X_j[j, ni - 1]]
            iref += [1, ni - 2]
            jref += [j, j]
    return (np.array(jj), np.array(ii), np.array(nx), np.array(ny), np.array(jref),
            np.array(iref))


def farfield_bc(grid, X, Y, f_new, g_new, gamma, rho_inf, u_inf, T_inf):
    """Equilibrium populations on the far-field nodes (Sec. III.A.2)."""
    jj, ii, nx, ny, jr, ir = farfield_nodes(grid, X, Y)
    inflow = (u_inf[0] * nx + u_inf[1] * ny) < 0.0
    rho_in, ux_in, uy_in, _, T_in = L.macroscopic(f_new[:, jr, ir], g_new[:, jr, ir], gamma)
    rho = np.where(inflow, rho_inf, rho_in)
    ux = np.where(inflow, u_inf[0], ux_in)
    uy = np.where(inflow, u_inf[1], uy_in)
    T = np.where(inflow, T_inf, T_in)
    fe, ge = L.equilibrium_populations(rho, ux, uy, T, gamma)
    f_new[:, jj, ii] = fe
    g_new[:, jj, ii] = ge
    return inflow
