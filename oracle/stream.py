"""ALE semi-Lagrangian streaming in float64 (paper Sec. II.A and II.B).
Test infrastructure only.

For every node and every velocity c_i, the rest velocity c_0 = 0 included:

1. transformed velocity  c^_i = g^{-1} (c_i - V_G), with g = dx/dX the
   Jacobian of the ALE map.  Reading of the printed "g^{-T} c_i - V_G": by the
   chain rule the advection velocity in the undeformed frame is
   (dx/dX)^{-1}(c - V_G) (the printed g^{-1} matrix is the inverse transpose of
   dx_k/dX_l, and V_G is a physical velocity).  g is taken at t^{n+1}:
   g = (dx^{n+1}/dxi)(dX/dxi)^{-1} from FE derivatives, V_G = (x^{n+1}-x^n)/dt.
2. departure point  X_dp = X - dt c^_i  (Sec. II.B, Eq. for X_dp),
3. its reference coordinates from the first-order (bilinear, 4-node) element
   map, solved by Newton among the cells that touch the node
   (Sec. II.B, Eq. for X_dp = sum_s X_s N'_s),
4. the population at the node is the second-order (9-node) Lagrange
   interpolant of the post-collision populations at the departure point
   (Sec. II.B, Eq. for f_i(X, t)).

The propagation holds for all nine populations.  The rest populations f_0,
g_0 do not move in physical space, but on a moving mesh their transformed
velocity c^_0 = -g^{-1} V_G is not zero, so they are interpolated at
X + dt g^{-1} V_G like the others (and are missing at a wall node whose point
lies in the body).  Where the mesh does not move (V_G = 0) the departure
point is the node itself, whose offsets are exactly zero, and the
interpolation returns the node's own value.

Reading for the structured mesh: the 9-node element is the 3 x 3 block of
nodes centred on the arriving node (shifted inward by one row on a wall or
far-field row, by one column on a C-grid exit column), with tensor-product
quadratic Lagrange shape functions of the offsets of xi_dp from the block
centre.  On a C-grid the block of a cut node reaches across the cut (row -1
is the mirrored row 1 of the other side).
"""

from __future__ import annotations

import numpy as np

from .lattice import CX, CY, Q


class CFLViolation(ValueError):
    """A departure point lies outside the cells that touch its node."""


# candidate cells touching a node, by the index offset of their lower-left corner
CANDIDATE_CELLS = ((-1, -1), (0, -1), (-1, 0), (0, 0))
CELL_TOL = 1e-12
# Reading (the paper does not say how a departure point on the wall line is
# classified): a wall node's departure point less than WALL_TOL (index units)
# below the wall line counts as on it, so it is interpolated, not missing.
# The tolerance makes the decision independent of rounding for points that
# lie on the wall line in exact arithmetic, such as those of populations
# moving along a straight slit at a junction with a body.
WALL_TOL = 1e-4


def bilinear_inverse(P00, P10, P01, P11, Px, Py, iters=60):
    """Solve X(s, t) = P for the bilinear map of one cell (Newton, float64).

    X(s, t) = P00 (1-s)(1-t) + P10 s (1-t) + P01 (1-s) t + P11 s t, with each
    corner a pair (x, y) of arrays.  Returns (s, t, residual).
    """
    s = np.full(np.shape(Px), 0.5)
    t = np.full(np.shape(Px), 0.5)
    for _ in range(iters):
        Xs = P00[0] * (1 - s) * (1 - t) + P10[0] * s * (1 - t) + P01[0] * (1 - s) * t + P11[0] * s * t
        Ys = P00[1] * (1 - s) * (1 - t) + P10[1] * s * (1 - t) + P01[1] * (1 - s) * t + P11[1] * s * t
        rx = Xs - Px
        ry = Ys - Py
        a_x = (P10[0] - P00[0]) * (1 - t) + (P11[0] - P01[0]) * t
        a_y = (P10[1] - P00[1]) * (1 - t) + (P11[1] - P01[1]) * t
        b_x = (P01[0] - P00[0]) * (1 - s) + (P11[0] - P10[0]) * s
        b_y = (P01[1] - P00[1]) * (1 - s) + (P11[1] - P10[1]) * s
        det = a_x * b_y - a_y * b_x
        ds = (b_y * rx - b_x * ry) / det
        dtt = (-a_y * rx + a_x * ry) / det
        with np.errstate(invalid="ignore"):
            s = s - ds
            t = t - dtt
            if np.all(~np.isfinite(ds) | (np.abs(ds) + np.abs(dtt) < 1e-15)):
                break
    Xs = P00[0] * (1 - s) * (1 - t) + P10[0] * s * (1 - t) + P01[0] * (1 - s) * t + P11[0] * s * t
    Ys = P00[1] * (1 - s) * (1 - t) + P10[1] * s * (1 - t) + P01[1] * (1 - s) * t + P11[1] * s * t
    return s, t, np.hypot(Xs - Px, Ys - Py)


def transformed_velocities(grid, X, Y, x1, y1, VGx, VGy):
    """c^_i = g^{-1}(c_i - V_G) for i = 0..8, with g = (dx^{n+1}/dxi)(dX/dxi)^{-1}.

    Returns a list of (c^x, c^y) pairs, one per velocity.
    """
    A = grid.metrics(x1, y1)            # x_xi, x_eta, y_xi, y_eta at t^{n+1}
    B = grid.metrics(X, Y)              # the same for the undeformed mesh
    # g = A B^{-1}
    detB = B[0] * B[3] - B[2] * B[1]
    Binv = (B[3] / detB, -B[1] / detB, -B[2] / detB, B[0] / detB)  # (11, 12, 21, 22)
    g11 = A[0] * Binv[0] + A[1] * Binv[2]
    g12 = A[0] * Binv[1] + A[1] * Binv[3]
    g21 = A[2] * Binv[0] + A[3] * Binv[2]
    g22 = A[2] * Binv[1] + A[3] * Binv[3]
    detg = g11 * g22 - g12 * g21
    out = []
    for i in range(Q):
        wx = CX[i] - VGx
        wy = CY[i] - VGy
        out.append(((g22 * wx - g12 * wy) / detg, (-g21 * wx + g11 * wy) / detg))
    return out


def departure_offsets(grid, X, Y, chx, chy, dt, wall_row=False):
    """Reference coordinates of X_dp = X - dt c^ relative to each node.

    Returns (a, b, missing): a, b are the index-space offsets of xi_dp from the
    node; ``missing`` marks departure points that leave the mesh through the
    wall (only when ``wall_row``): wall nodes search only the cells above the
    wall, and a point more than WALL_TOL below them lies in the body (for
    those a is NaN and b the offset below the wall line).  Raises
    CFLViolation if a departure point lies in none of the cells touching its
    node.
    """
    Pdx = -dt * chx                      # X_dp - X, relative to the node
    Pdy = -dt * chy
    # a departure point on the node itself (a rest population where the mesh
    # does not move) is a corner of every cell round the node: offsets 0
    at_node = (Pdx == 0.0) & (Pdy == 0.0)
    a = np.full(X.shape, np.nan)
    b = np.full(X.shape, np.nan)
    found = np.zeros(X.shape, dtype=bool)
    missing = np.zeros(X.shape, dtype=bool)
    wall_node = (grid.jj == 0) & grid.wall_col[None, :] if wall_row else np.zeros(X.shape, bool)
    for (di0, dj0) in CANDIDATE_CELLS:
        corners = []
        for (ci, cj) in ((0, 0), (1, 0), (0, 1), (1, 1)):
            px, py = grid.neighbour_pos(X, Y, di0 + ci, dj0 + cj)
            if dj0 < 0:                     # no cells below the wall
                px = np.where(wall_node, np.nan, px)
            corners.append((px - X, py - Y))
        with np.errstate(invalid="ignore", divide="ignore"):
            s, t, _ = bilinear_inverse(*corners, Pdx, Pdy)
        t_lo = np.where(wall_node, -WALL_TOL, -CELL_TOL) if dj0 == 0 else -CELL_TOL
        inside = ((s >= -CELL_TOL) & (s <= 1 + CELL_TOL)
                  & (t >= t_lo) & (t <= 1 + CELL_TOL))
        take = inside & ~found
        a = np.where(take, di0 + s, a)
        b = np.where(take, dj0 + t, b)
        found |= take
        if wall_row and dj0 == 0:
            # a wall-node departure point below the first cell row lies in the body
            below = ((s >= -CELL_TOL) & (s <= 1 + CELL_TOL) & (t < -WALL_TOL) & wall_node)
            new = below & ~found & ~missing
            b = np.where(new, t, b)
            missing |= new
    missing &= ~found
    a = np.where(at_node, 0.0, a)
    b = np.where(at_node, 0.0, b)
    found |= at_node
    missing &= ~at_node
    bad = ~found & ~missing
    if np.any(bad):
        k = int(np.flatnonzero(bad.ravel())[0])
        raise CFLViolation(f"departure point outside the node's cells at flat node {k}")
    return a, b, missing


def lagrange_1d(p, a):
    """Quadratic Lagrange basis on the nodes {-1, 0, +1}: L_p(a) =
    prod_{m != p} (a - m) / (p - m)."""
    out = np.ones_like(a)
    for m in (-1, 0, 1):
        if m != p:
            out = out * (a - m) / (p - m)
    return out


def stencil_centres(grid):
    """Index-space centre (ic, jc) of every node's 3 x 3 element: the node
    itself, moved inward by one row on a wall or far-field row and by one
    column on a C-grid exit column."""
    ic = grid.ii.copy()
    jc = grid.jj.copy()
    if not grid.periodic_j:
        jc[0] = np.where(grid.wall_col, 1, 0)
        jc[-1] = grid.nj - 2
    if grid.cgrid:
        ic[:, 0] = 1
        ic[:, -1] = grid.ni - 2
    return ic, jc


def interpolate(grid, fstar_i, a, b):
    """f_i(node) = sum_s N_s(xi_dp) f*_i(xi_s) over the 3 x 3 element
    (Sec. II.B, Eq. for f_i(X, t))."""
    ic, jc = stencil_centres(grid)
    ac = a + (grid.ii - ic)
    bc = b + (grid.jj - jc)
    out = np.zeros(a.shape)
    for p in (-1, 0, 1):
        La = lagrange_1d(p, ac)
        for q in (-1, 0, 1):
            Lb = lagrange_1d(q, bc)
            out = out + La * Lb * grid.gather(fstar_i, ic + p, jc + q)
    return out


def boundary_nodes(grid):
    """Nodes whose populations the far-field condition replaces: row nj - 1
    of an O-grid or C-grid, and the two exit columns of a C-grid."""
    far = np.zeros((grid.nj, grid.ni), dtype=bool)
    if not grid.periodic_j:
        far[-1] = True
    if grid.cgrid:
        far[:, 0] = True
        far[:, -1] = True
    return far


def stream(grid, X, Y, x1, y1, VGx, VGy, dt, fpost, gpost):
    """Interpolating ALE streaming of both population sets.

    Returns (f_new, g_new, missing[9]); far-field nodes (whose populations the
    boundary condition replaces) are left NaN, as are populations flagged
    missing at the wall.
    """
    chat = transformed_velocities(grid, X, Y, x1, y1, VGx, VGy)
    f_new = np.full(fpost.shape, np.nan)
    g_new = np.full(gpost.shape, np.nan)
    missing = np.zeros(fpost.shape, dtype=bool)
    active = ~boundary_nodes(grid)
    wall = bool(np.any(grid.wall_col))
    for i in range(Q):
        chx, chy = chat[i]
        # far-field nodes get a zero offset (never used) so they cannot raise
        chx = np.where(active, chx, 0.0)
        chy = np.where(active, chy, 0.0)
        a, b, miss = departure_offsets(grid, X, Y, chx, chy, dt, wall_row=wall)
        a = np.where(np.isnan(a), 0.0, a)
        b = np.where(np.isnan(b), 0.0, b)
        fi = interpolate(grid, fpost[i], a, b)
        gi = interpolate(grid, gpost[i], a, b)
        keep = active & ~miss
        f_new[i] = np.where(keep, fi, np.nan)
        g_new[i] = np.where(keep, gi, np.nan)
        missing[i] = miss & active
    return f_new, g_new, missing
