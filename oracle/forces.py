"""Surface force and moment in float64 (paper Sec. III, force on wall
elements).  Test infrastructure only.

At every wall node k:
    sigma_k = -p I - (1 - omega/2) P^(1),   P^(1) = sum_i (f_i - f_i^eq) c_i c_i
    F_k     = sigma_k . (n ds)_k
with (n ds)_k = 1/2 rot_{+90}(x_{k+1} - x_{k-1}), the node-lumped normal of
the two half wall segments adjacent to the node, pointing out of the body
into the fluid.  (Reading: the paper sums element forces; lumping each
element's two end-node contributions onto the nodes gives this trapezoid
form, and the lumped normals of a closed wall sum to zero exactly.)
F = sum_k F_k and M_EA = sum_k (x_k - x_EA) x F_k, both summed in node order.

The wall polygon of a body is the closed sequence of its distinct wall
nodes: the whole row j = 0 of an O-grid; on a C-grid the columns from the
lower trailing-edge copy up to, not including, the upper copy (the same
point), and on a twin O-grid the columns of the body's wall segment without
its second junction copy, so that the neighbours k +- 1 run cyclically round
the body.
"""

from __future__ import annotations

import numpy as np

from . import lattice as L


def wall_polygon(grid, seg=0):
    """Columns of the distinct wall nodes of wall segment `seg` (body `seg`)
    in polygon order."""
    i0, n, dup = grid.segments[seg]
    return np.arange(i0, i0 + n - (1 if dup else 0))


def wall_lumped_normals(grid, x, y, seg=0):
    """(n ds)_k for the wall polygon's nodes, from their cyclic neighbours."""
    cols = wall_polygon(grid, seg)
    px, py = x[0, cols], y[0, cols]
    tx = 0.5 * (np.roll(px, -1) - np.roll(px, 1))
    ty = 0.5 * (np.roll(py, -1) - np.roll(py, 1))
    return cols, -ty, tx


def wall_stress(f0, g0, gamma, mu, Pr, dt):
    """sigma = -p I - (1 - omega/2) P^(1) at wall nodes from populations [9, ni]."""
    rho, ux, uy, E, T = L.macroscopic(f0, g0, gamma)
    fe = L.feq(rho, ux, uy, T)
    P1xx = np.zeros_like(rho)
    P1xy = np.zeros_like(rho)
    P1yy = np.zeros_like(rho)
    for i in range(L.Q):
        d = f0[i] - fe[i]
        P1xx = P1xx + d * L.CX[i] * L.CX[i]
        P1xy = P1xy + d * L.CX[i] * L.CY[i]
        P1yy = P1yy + d * L.CY[i] * L.CY[i]
    omega, _ = L.relaxation_rates(rho, T, mu, Pr, dt)
    p = rho * T
    k = 1.0 - 0.5 * omega
    return -p - k * P1xx, -k * P1xy, -p - k * P1yy


def wall_force(grid, f, g, x, y, gamma, mu, Pr, dt, ea_pos, seg=0):
    """Total (F_x, F_y, M_EA) on the wall of body `seg`; ea_pos is the
    physical position of the elastic axis (about which the moment is taken)
    at the same time level as (x, y)."""
    cols, nx, ny = wall_lumped_normals(grid, x, y, seg)
    sxx, sxy, syy = wall_stress(f[:, 0, cols], g[:, 0, cols], gamma, mu, Pr, dt)
    Fx_k = sxx * nx + sxy * ny
    Fy_k = sxy * nx + syy * ny
    rx = x[0, cols] - ea_pos[0]
    ry = y[0, cols] - ea_pos[1]
    Mz_k = rx * Fy_k - ry * Fx_k
    Fx = 0.0
    Fy = 0.0
    Mz = 0.0
    for k in range(cols.size):
        Fx += Fx_k[k]
        Fy += Fy_k[k]
        Mz += Mz_k[k]
    return Fx, Fy, Mz
