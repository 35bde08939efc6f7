"""Structured-mesh geometry for the oracle: neighbour access, finite-element
first derivatives, physical gradients, and blending-function mesh motion.
Test infrastructure only.

Fields are arrays [nj, ni] on node (i, j), i fastest.

Gradients (Sec. II.B, FE derivative d_X C = J^{-1} sum_s C_s d_xi N_s): at a
node of the structured mesh the derivative of the quadratic Lagrange element
centred on that node is the centred difference (C_{+1} - C_{-1}) / 2 in index
space; on a non-periodic end row the element is one-sided and its derivative
at the end node is (-3 C_0 + 4 C_1 - C_2) / 2.  Physical derivatives follow
from the chain rule with the mesh metrics computed the same way (Sec. II.B,
J^{-1} and det J).
"""

from __future__ import annotations

import numpy as np

TOPO_PERIODIC2 = 0
TOPO_OGRID = 1
TOPO_CGRID = 2
TOPO_TWIN = 3


class Grid:
    """Index topology of a structured mesh.

    periodic_i / periodic_j: wrap in that index.  shift_i / shift_j: vectors
    added to coordinates when a neighbour is taken across the periodic seam
    (zero for an O-grid's azimuthal seam, the period for a doubly periodic box).

    Cut topologies (a C-grid, a twin O-grid): part of row j = 0 is a cut
    across which node (i, -m) is node (mirror(i), m), mirror(i) = M - i
    (mod ni on a twin O-grid).  The cut columns are the "primary" columns
    cut_a < i < cut_b and their mirror images; every other column of row 0 is
    a wall column.  C-grid: i is not periodic (columns 0 and ni - 1 are the
    exit boundary), M = ni - 1, primary columns 0 .. n_wake - 1, and the wall
    columns [n_wake, ni - n_wake) include both trailing-edge copies.  Twin
    O-grid: i periodic, nA = ni - 2 n_wake - n_wall2, M = nA, primary columns
    nA < i < nA + n_wake (one side of the slit); the walls are the columns
    [0, nA] of the first body and [nA + n_wake, nA + n_wake + n_wall2] of the
    second, each with its junction point twice.  An O-grid's wall is the
    whole row.

    ``segments``: the walls as (first column, columns, duplicated end), the
    last column of a segment with a duplicated end being the same point as
    its first; segment k is the wall of body k.
    """

    def __init__(self, ni, nj, topo, shift_i=(0.0, 0.0), shift_j=(0.0, 0.0), n_wake=0,
                 n_wall2=0):
        self.ni, self.nj, self.topo = int(ni), int(nj), int(topo)
        self.cgrid = self.topo == TOPO_CGRID
        self.twin = self.topo == TOPO_TWIN
        self.cut = self.cgrid or self.twin
        self.periodic_i = not self.cgrid
        self.periodic_j = self.topo == TOPO_PERIODIC2
        self.n_wake = int(n_wake) if self.cut else 0
        self.shift_i = np.asarray(shift_i, dtype=np.float64)
        self.shift_j = np.asarray(shift_j, dtype=np.float64)
        self.jj, self.ii = np.meshgrid(np.arange(self.nj), np.arange(self.ni),
                                       indexing="ij")
        cols = np.arange(self.ni)
        if self.cgrid:
            self.cut_a, self.cut_b, self.M = -1, self.n_wake, self.ni - 1
            self.segments = [(self.n_wake, self.ni - 2 * self.n_wake, True)]
        elif self.twin:
            nB = int(n_wall2)
            nA = self.ni - 2 * self.n_wake - nB
            self.cut_a, self.cut_b, self.M = nA, nA + self.n_wake, nA
            self.segments = [(0, nA + 1, True), (nA + self.n_wake, nB + 1, True)]
        else:
            self.cut_a = self.cut_b = self.M = 0
            self.segments = [] if self.periodic_j else [(0, self.ni, False)]
        if self.cut:
            prim = (cols > self.cut_a) & (cols < self.cut_b)
            self.cut_col = prim | prim[self.mirror(cols)]
            self.primary_cols = cols[prim]
            self.wall_col = ~self.cut_col
        else:
            self.cut_col = np.zeros(self.ni, dtype=bool)
            self.primary_cols = cols[:0]
            self.wall_col = np.full(self.ni, not self.periodic_j)

    def mirror(self, i):
        """Column of the node across the cut from column i."""
        m = self.M - np.asarray(i)
        return m % self.ni if self.periodic_i else m

    @classmethod
    def from_mesh(cls, mesh):
        return cls(mesh.ni, mesh.nj, mesh.topo, mesh.shift_i, mesh.shift_j,
                   getattr(mesh, "n_wake", 0), getattr(mesh, "n_wall2", 0))

    # ---- neighbour access -------------------------------------------------
    def node_index(self, ii, jj):
        """Storage indices (i, j) of index-space positions (ii, jj), and whether
        that node exists: wrap in periodic indices, mirror across the C-grid
        cut for jj < 0."""
        ii = np.asarray(ii)
        jj = np.asarray(jj)
        valid = np.ones(np.broadcast(ii, jj).shape, dtype=bool)
        if self.cut:
            below = jj < 0
            ii = np.where(below, self.M - ii, ii)
            jj = np.where(below, -jj, jj)
        if self.periodic_i:
            ii = ii % self.ni
        else:
            valid &= (ii >= 0) & (ii < self.ni)
        if self.periodic_j:
            jj = jj % self.nj
        else:
            valid &= (jj >= 0) & (jj < self.nj)
        return np.clip(ii, 0, self.ni - 1), np.clip(jj, 0, self.nj - 1), valid

    def gather(self, F, ii, jj):
        """F at index-space positions (ii, jj); NaN where no node exists."""
        si, sj, valid = self.node_index(ii, jj)
        return np.where(valid, F[sj, si].astype(np.float64), np.nan)

    def neighbour(self, F, di, dj):
        """F at (i + di, j + dj); NaN where the neighbour does not exist."""
        return self.gather(F, self.ii + di, self.jj + dj)

    def neighbour_pos(self, X, Y, di, dj):
        """Coordinates of node (i + di, j + dj) as seen from node (i, j), with
        the periodic shift applied across a seam."""
        xs = self.neighbour(X, di, dj)
        ys = self.neighbour(Y, di, dj)
        if self.periodic_i:
            wrap_i = np.floor_divide(self.ii + di, self.ni)
            xs = xs + wrap_i * self.shift_i[0]
            ys = ys + wrap_i * self.shift_i[1]
        if self.periodic_j:
            wrap_j = np.floor_divide(self.jj + dj, self.nj)
            xs = xs + wrap_j * self.shift_j[0]
            ys = ys + wrap_j * self.shift_j[1]
        return xs, ys

    # ---- index-space derivatives -------------------------------------------
    def d_i(self, F):
        """dF/d(i): centred, one-sided 3-point on the C-grid exit columns."""
        if self.periodic_i:
            return 0.5 * (self.neighbour(F, 1, 0) - self.neighbour(F, -1, 0))
        out = np.empty_like(F, dtype=np.float64)
        out[:, 1:-1] = 0.5 * (F[:, 2:] - F[:, :-2])
        out[:, 0] = 0.5 * (-3.0 * F[:, 0] + 4.0 * F[:, 1] - F[:, 2])
        out[:, -1] = 0.5 * (3.0 * F[:, -1] - 4.0 * F[:, -2] + F[:, -3])
        return out

    def d_j(self, F):
        """dF/d(j): centred inside (and across the C-grid cut), one-sided
        3-point on the wall row and on the far-field row."""
        if self.periodic_j:
            return 0.5 * (self.neighbour(F, 0, 1) - self.neighbour(F, 0, -1))
        out = np.empty_like(F, dtype=np.float64)
        out[1:-1] = 0.5 * (F[2:] - F[:-2])
        out[0] = 0.5 * (-3.0 * F[0] + 4.0 * F[1] - F[2])
        out[-1] = 0.5 * (3.0 * F[-1] - 4.0 * F[-2] + F[-3])
        if self.cut:
            mirror = F[1, self.mirror(np.arange(self.ni))]
            out[0] = np.where(self.cut_col, 0.5 * (F[1] - mirror), out[0])
        return out

    def metrics(self, x, y):
        """(x_xi, x_eta, y_xi, y_eta) of a coordinate field, with seams shifted."""
        if self.cut:
            return self.d_i(x), self.d_j(x), self.d_i(y), self.d_j(y)
        xp, yp = self.neighbour_pos(x, y, 1, 0)
        xm, ym = self.neighbour_pos(x, y, -1, 0)
        x_xi = 0.5 * (xp - xm)
        y_xi = 0.5 * (yp - ym)
        if self.periodic_j:
            xp, yp = self.neighbour_pos(x, y, 0, 1)
            xm, ym = self.neighbour_pos(x, y, 0, -1)
            x_eta = 0.5 * (xp - xm)
            y_eta = 0.5 * (yp - ym)
        else:
            x_eta = self.d_j(x)
            y_eta = self.d_j(y)
        return x_xi, x_eta, y_xi, y_eta

    def grad(self, C, x, y):
        """Physical gradient (dC/dx, dC/dy) on the mesh with coordinates (x, y):

            dC/dx = ( y_eta C_xi - y_xi C_eta) / det J
            dC/dy = (-x_eta C_xi + x_xi C_eta) / det J
            det J = x_xi y_eta - y_xi x_eta           (Sec. II.B)
        """
        x_xi, x_eta, y_xi, y_eta = self.metrics(x, y)
        det = x_xi * y_eta - y_xi * x_eta
        C_xi = self.d_i(C)
        C_eta = self.d_j(C)
        return ((y_eta * C_xi - y_xi * C_eta) / det,
                (-x_eta * C_xi + x_xi * C_eta) / det)


# ---- blending-function mesh motion (Sec. II.D) ------------------------------

def r5(s):
    """Fifth-order blending polynomial r_5(s) = 10 s^3 - 15 s^4 + 6 s^5."""
    return 10.0 * s ** 3 - 15.0 * s ** 4 + 6.0 * s ** 5


def distance_to_wall(X, Y, px, py):
    """Euclidean distance from each point (X, Y) to the closed polygon with
    vertices (px, py): the minimum over its edges of the point-segment
    distance (brute force, row by row)."""
    ax, ay = np.asarray(px, dtype=np.float64), np.asarray(py, dtype=np.float64)
    ex, ey = np.roll(ax, -1) - ax, np.roll(ay, -1) - ay
    ee = ex * ex + ey * ey
    out = np.empty(X.shape)
    for j in range(X.shape[0]):
        x = X[j][:, None]
        y = Y[j][:, None]
        t = np.clip(((x - ax) * ex + (y - ay) * ey) / ee, 0.0, 1.0)
        dx = x - (ax + t * ex)
        dy = y - (ay + t * ey)
        out[j] = np.sqrt(np.min(dx * dx + dy * dy, axis=1))
    return out


def blend_factor(X, Y, body, wall=None):
    """r_blend: 0 inside the rigid region, 1 beyond the blend region, r_5 of
    the normalised position in between (Sec. II.D).  The position is the
    radial distance from the body's blending centre in the undeformed frame,
    or, for blend_mode 1 (the distance-field variant the paper suggests for
    slender bodies), the distance to the wall polygon `wall` = (px, py)."""
    if getattr(body, "blend_mode", 0) == 1:
        d = distance_to_wall(X, Y, wall[0], wall[1])
    else:
        d = np.hypot(X - body.center[0], Y - body.center[1])
    s = (d - body.r_rigid) / (body.r_blend - body.r_rigid)
    return np.where(s < 0.0, 0.0, np.where(s > 1.0, 1.0, r5(np.clip(s, 0.0, 1.0))))


def rigid_map(X, Y, body, h, alpha):
    """G'_x(X): rigid motion of the body, translation h along y and a
    counter-clockwise rotation alpha about the elastic axis."""
    ex, ey = body.ea
    c, s = np.cos(alpha), np.sin(alpha)
    dx = X - ex
    dy = Y - ey
    return ex + c * dx - s * dy, ey + h + s * dx + c * dy


def rigid_displacement(X, Y, body, h, alpha):
    """G'_x(X) - X = (0, h) + (R(alpha) - I)(X - X_EA), evaluated without
    forming G' so that a body at rest gives exactly zero."""
    ex, ey = body.ea
    c, s = np.cos(alpha), np.sin(alpha)
    dx = X - ex
    dy = Y - ey
    return (c - 1.0) * dx - s * dy, h + s * dx + (c - 1.0) * dy


def master_of(bodies, k):
    """Index of the body whose rigid motion body k follows: itself, or the
    body it is linked to (a rigid assembly with one set of degrees of
    freedom)."""
    link = getattr(bodies[k], "link", -1)
    return k if link < 0 else link


def blend_factors(X, Y, bodies, walls=None):
    """r_blend of every body (list of arrays).  Each body has its own region
    of influence; the regions may not overlap (Sec. II.D, several bodies):
    asserted here, node by node, as at most one body with r < 1."""
    walls = walls if walls is not None else [None] * len(bodies)
    r = [blend_factor(X, Y, b, w) for b, w in zip(bodies, walls)]
    if len(r) > 1:
        inside = np.sum([rk < 1.0 for rk in r], axis=0)
        assert np.all(inside <= 1), "regions of influence overlap"
    return r


def deformed_positions(X, Y, bodies, states, wall=None, r=None):
    """x = r_blend X + (1 - r_blend) G'_x(X, t) (Sec. II.D), evaluated as
    x = X + (1 - r_blend)(G'_x(X) - X), which is the same expression.  With
    several bodies every body moves the nodes of its own region of influence:
    x = X + sum_k (1 - r_k)(G'_k(X) - X), at most one term being non-zero at a
    node; G'_k of a linked body is the rigid map (elastic axis and state) of
    the body it is linked to.

    ``states`` holds (h, alpha, hdot, alphadot) per body.  With no body x = X.
    ``wall``: the wall polygon (px, py) of the body (one body) or the list of
    polygons (one per body), used by distance blending.  ``r``: the blending
    factor(s) if already known (they depend on the undeformed mesh only).
    """
    if not bodies:
        return X.copy(), Y.copy()
    if wall is not None and len(bodies) == 1 and not isinstance(wall, list):
        wall = [wall]
    if r is None:
        r = blend_factors(X, Y, bodies, wall)
    elif not isinstance(r, list):
        r = [r]
    dx = np.zeros_like(X, dtype=np.float64)
    dy = np.zeros_like(Y, dtype=np.float64)
    for k in range(len(bodies)):
        m = master_of(bodies, k)
        ux, uy = rigid_displacement(X, Y, bodies[m], states[m][0], states[m][1])
        dx = dx + (1.0 - r[k]) * ux
        dy = dy + (1.0 - r[k]) * uy
    return X + dx, Y + dy
