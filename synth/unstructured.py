"""Unstructured second-order quadrilateral meshes (9-node elements) on a
periodic box, as input data: node coordinates and element connectivity only.

The paper's own discretisation uses unstructured second-order finite-element
meshes.  This generator makes genuinely unstructured ones without an external
mesher: a periodic m x m square grid is split into triangles (one diagonal per
square, alternating with a seeded coin), every triangle is split into three
quadrilaterals through its edge midpoints and centroid, and every
quadrilateral becomes a 9-node element by adding its edge midpoints (shared
with the neighbour) and its centre.  Vertices of the grid meet 4 to 8
quadrilaterals, triangle centroids 3, edge midpoints 4.  The element corners
are then displaced by a smooth periodic field, the edge and centre nodes put
where the corners' bilinear map places them (straight-sided elements), and
the nodes renumbered along a space-filling (Morton) order.

Element node order: corners at local (-1,-1), (1,-1), (1,1), (-1,1), then the
edge midpoints (0,-1), (1,0), (0,1), (-1,0), then the centre (0,0), counter-
clockwise (positive Jacobian).  Elements crossing the periodic seams carry,
for each of their nodes, the number of periods (sx, sy) to add to that node's
stored coordinates to place it next to the element's other nodes.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# local (xi, eta) of the 9 element nodes, in element node order
Q9_LOCAL = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1],
                     [0, -1], [1, 0], [0, 1], [-1, 0], [0, 0]], dtype=np.int64)


@dataclass
class UnstructuredMesh:
    X: np.ndarray            # [N] float64
    Y: np.ndarray            # [N] float64
    elems: np.ndarray        # [E, 9] int32 node indices
    shifts: np.ndarray       # [E, 9, 2] int8 periods added to each element node
    period: tuple            # (Lx, Ly); (0, 0) for a bounded mesh
    info: dict = field(default_factory=dict)
    wall_nodes: np.ndarray | None = None   # [n] body polygon, clockwise (bounded meshes)
    far_nodes: np.ndarray | None = None    # [m] outer boundary (bounded meshes)

    @property
    def n_nodes(self) -> int:
        return int(self.X.size)

    @property
    def n_elems(self) -> int:
        return int(self.elems.shape[0])

    # the library's mesh description: topology 4, ni = nodes, nj = 1, the
    # periods as the seam shifts
    topo = 4
    nj = 1

    @property
    def ni(self) -> int:
        return self.n_nodes

    @property
    def shift_i(self):
        return (float(self.period[0]), 0.0)

    @property
    def shift_j(self):
        return (0.0, float(self.period[1]))

    def interleaved(self) -> np.ndarray:
        return np.stack([self.X, self.Y], axis=-1)[None]


def _morton(ix, iy, bits=16):
    out = np.zeros_like(ix, dtype=np.int64)
    for b in range(bits):
        out |= ((ix >> b) & 1) << (2 * b)
        out |= ((iy >> b) & 1) << (2 * b + 1)
    return out


def unstructured_q9_mesh(m: int = 32, L: float | None = None, amp: float = 0.06,
                         seed: int = 0) -> UnstructuredMesh:
    """Periodic box [0, L)^2 (L = 6 m by default, so that the smallest node
    spacing is about one lattice unit), 6 m^2 elements, 24 m^2 nodes.

    amp: amplitude of the smooth displacement, in units of the grid spacing
    L / m (x += amp h sin(2 pi y / L) sin(2 pi x / L + 1), y += amp h
    sin(2 pi x / L) cos(2 pi y / L + 2))."""
    L = float(6 * m if L is None else L)
    h = L / m
    rng = np.random.default_rng(seed)
    # exact positions in units of h/24 (integers): grid points are multiples
    # of 24, triangle edge midpoints of 12, centroids of 8, and the element
    # edge midpoints and centres built from them stay integral
    S = 24 * m                                  # period in lattice units
    key_to_id = {}
    pts = []

    def node(px, py):
        k = (px % S, py % S)
        i = key_to_id.get(k)
        if i is None:
            i = len(pts)
            key_to_id[k] = i
            pts.append(k)
        return i

    elems = []
    shifts = []

    def add_quad(c):
        # c: 4 corners (unwrapped lattice coordinates), counter-clockwise
        mids = [((c[a][0] + c[b][0]) // 2, (c[a][1] + c[b][1]) // 2)
                for a, b in ((0, 1), (1, 2), (2, 3), (3, 0))]
        cen = (sum(p[0] for p in c) // 4, sum(p[1] for p in c) // 4)
        allp = list(c) + mids + [cen]
        ids = [node(*p) for p in allp]
        sh = [((p[0] - (p[0] % S)) // S, (p[1] - (p[1] % S)) // S) for p in allp]
        elems.append(ids)
        shifts.append(sh)

    for j in range(m):
        for i in range(m):
            x0, y0 = 24 * i, 24 * j
            A, B, C, D = (x0, y0), (x0 + 24, y0), (x0 + 24, y0 + 24), (x0, y0 + 24)
            tris = [(A, B, C), (A, C, D)] if rng.random() < 0.5 else [(A, B, D), (B, C, D)]
            for (p, q, r) in tris:
                g = ((p[0] + q[0] + r[0]) // 3, (p[1] + q[1] + r[1]) // 3)
                mpq = ((p[0] + q[0]) // 2, (p[1] + q[1]) // 2)
                mqr = ((q[0] + r[0]) // 2, (q[1] + r[1]) // 2)
                mrp = ((r[0] + p[0]) // 2, (r[1] + p[1]) // 2)
                add_quad([p, mpq, g, mrp])
                add_quad([q, mqr, g, mpq])
                add_quad([r, mrp, g, mqr])
    P = np.array(pts, dtype=np.int64)
    E = np.array(elems, dtype=np.int64)
    SH = np.array(shifts, dtype=np.int64)
    # lattice units -> length; the smooth periodic displacement moves the
    # element corners, and the edge and centre nodes are then placed where
    # the corners' bilinear map puts them (straight-sided elements, as a
    # second-order mesher makes away from curved boundaries)
    x = P[:, 0] * (L / S)
    y = P[:, 1] * (L / S)
    tx, ty = 2 * np.pi * x / L, 2 * np.pi * y / L
    X = x + amp * h * np.sin(ty) * np.sin(tx + 1.0)
    Y = y + amp * h * np.sin(tx) * np.cos(ty + 2.0)
    ex = X[E] + SH[..., 0] * L
    ey = Y[E] + SH[..., 1] * L
    for k, (a, b) in enumerate(((0, 1), (1, 2), (2, 3), (3, 0))):
        X[E[:, 4 + k]] = 0.5 * (ex[:, a] + ex[:, b]) - SH[:, 4 + k, 0] * L
        Y[E[:, 4 + k]] = 0.5 * (ey[:, a] + ey[:, b]) - SH[:, 4 + k, 1] * L
    X[E[:, 8]] = 0.25 * (ex[:, 0] + ex[:, 1] + ex[:, 2] + ex[:, 3]) - SH[:, 8, 0] * L
    Y[E[:, 8]] = 0.25 * (ey[:, 0] + ey[:, 1] + ey[:, 2] + ey[:, 3]) - SH[:, 8, 1] * L
    # Morton renumbering of the nodes
    order = np.argsort(_morton(P[:, 0], P[:, 1]), kind="stable")
    new_id = np.empty_like(order)
    new_id[order] = np.arange(order.size)
    X, Y = X[order], Y[order]
    E = new_id[E]
    # elements in Morton order of their centre node
    eorder = np.argsort(E[:, 8], kind="stable")
    E, SH = E[eorder], SH[eorder]
    return UnstructuredMesh(X.astype(np.float64), Y.astype(np.float64), E.astype(np.int32),
                            SH.astype(np.int8), (L, L),
                            info={"kind": "tri_split_q9", "m": m, "amp": amp, "seed": seed})


def element_coords(mesh: UnstructuredMesh):
    """Unwrapped coordinates [E, 9] of every element's nodes."""
    ex = mesh.X[mesh.elems] + mesh.shifts[..., 0] * mesh.period[0]
    ey = mesh.Y[mesh.elems] + mesh.shifts[..., 1] * mesh.period[1]
    return ex, ey


def smallest_patch_reach(mesh: UnstructuredMesh) -> float:
    """A lower bound on how far a departure point may move from its node and
    stay inside the node's elements: over all elements, the smallest distance
    from one of its nodes to an edge of the element that does not hold that
    node, halved (a node's elements surround it at least that far)."""
    ex, ey = element_coords(mesh)
    corners = [(0, 1), (1, 2), (2, 3), (3, 0)]
    best = np.inf
    for a in range(9):
        for (p, q) in corners:
            # skip edges that contain node a (corners p, q or the midpoint between them)
            mid = 4 + corners.index((p, q))
            if a in (p, q, mid):
                continue
            x1, y1, x2, y2 = ex[:, p], ey[:, p], ex[:, q], ey[:, q]
            tx, ty = x2 - x1, y2 - y1
            d = np.abs((ex[:, a] - x1) * ty - (ey[:, a] - y1) * tx) / np.hypot(tx, ty)
            best = min(best, float(d.min()))
    return 0.5 * best


def unstructured_pulse_case(m: int = 16, amp: float = 0.06, seed: int = 0, Ma: float = 0.1,
                            nu: float = 0.02, pulse: float = 1e-3, T0: float = 1.0 / 3.0,
                            gamma: float = 1.4, Pr: float = 0.71, storage: int = 0):
    """Gas streaming diagonally through the periodic unstructured box with a
    Gaussian density pulse (width 4 lattice units) at the centre.  dt is a
    third of the smallest patch reach divided by sqrt(2), so every departure
    point stays inside its node's elements."""
    from .configs import FluidParams, sound_speed
    mesh = unstructured_q9_mesh(m, amp=amp, seed=seed)
    dt = smallest_patch_reach(mesh) / (3.0 * np.sqrt(2.0))
    U = Ma * sound_speed(gamma, T0)
    u0 = (U / np.sqrt(2.0), U / np.sqrt(2.0))
    fluid = FluidParams(gamma=gamma, Pr=Pr, mu=nu, rho_inf=1.0, T_inf=T0, u_inf=u0, dt=dt,
                        storage=storage)
    Lx, Ly = mesh.period
    dx = mesh.X - 0.5 * Lx
    dy = mesh.Y - 0.5 * Ly
    dx -= Lx * np.round(dx / Lx)
    dy -= Ly * np.round(dy / Ly)
    rho = 1.0 + pulse * np.exp(-(dx * dx + dy * dy) / (2.0 * 16.0))
    N = mesh.n_nodes
    return mesh, fluid, (rho, np.full(N, u0[0]), np.full(N, u0[1]), np.full(N, T0))


def cylinder_q9_mesh(n_theta: int = 64, D: float = 80.0, far_D: float = 8.0, seed: int = 0,
                     center=(0.0, 0.0), mirror: bool = False, quarter_turn: bool = False) -> UnstructuredMesh:
    """Unstructured 9-node quadrilateral mesh of the annulus between a
    cylinder of diameter D and a circle of far_D * D, as input data: the
    annulus is cut into n_theta x n_r cells of a polar grid (square cells:
    radii growing by 1 + 2 pi / n_theta), every cell into two triangles by a
    seeded diagonal, every triangle into three quadrilaterals through its edge
    midpoints and centroid, all in physical coordinates (straight-sided
    elements; the wall is the polygon through the grid's wall points, with
    the element edge nodes on its chords).  Nodes renumbered in Morton order
    of their coordinates, elements by their centre node.

    mirror (n_theta even): the lower half is the mirror image of the upper
    half about the x axis through the centre (diagonals mirrored, corner
    coordinates mirrored exactly).  quarter_turn: the mesh turned by +90
    degrees about the centre (a mirrored mesh is then symmetric about the y
    axis through the centre).

    Also returns, on the mesh: `wall_nodes`, the nodes on the body polygon
    in clockwise order (a rotation by +90 degrees of the polygon's tangent
    points into the fluid), and `far_nodes`, the nodes on the outer circle."""
    rng = np.random.default_rng(seed)
    R = 0.5 * D
    q = 1.0 + 2.0 * np.pi / n_theta
    n_r = int(np.ceil(np.log(far_D * D / D) / np.log(q)))
    S = 24 * n_theta                                   # index-space period along theta

    def corner(i, j):
        i = i % n_theta
        r = R * q ** j
        if mirror and 2 * i > n_theta:
            x, y = corner(n_theta - i, j)
            return (x, 2.0 * center[1] - y)
        t = 2.0 * np.pi * i / n_theta
        return (center[0] + r * np.cos(t), center[1] + r * np.sin(t))

    if mirror and n_theta % 2:
        raise ValueError("a mirrored mesh needs an even n_theta")

    key_to_id = {}
    pos = []

    def node(key, p):
        k = (key[0] % S, key[1])
        i = key_to_id.get(k)
        if i is None:
            i = len(pos)
            key_to_id[k] = i
            pos.append(p)
        return i

    elems = []

    def mid(a, b):
        return ((a[0] + b[0]) // 2, (a[1] + b[1]) // 2)

    def pmid(a, b):
        return (0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]))

    def add_quad(keys, pts):
        # keys / pts: 4 corners; orient counter-clockwise in physical space
        area = 0.5 * sum(pts[c][0] * pts[(c + 1) % 4][1] - pts[(c + 1) % 4][0] * pts[c][1]
                         for c in range(4))
        if area < 0:
            keys = [keys[0], keys[3], keys[2], keys[1]]
            pts = [pts[0], pts[3], pts[2], pts[1]]
        ids = [node(keys[c], pts[c]) for c in range(4)]
        for a, b in ((0, 1), (1, 2), (2, 3), (3, 0)):
            ids.append(node(mid(keys[a], keys[b]), pmid(pts[a], pts[b])))
        ck = (sum(k[0] for k in keys) // 4, sum(k[1] for k in keys) // 4)
        ids.append(node(ck, (0.25 * sum(p[0] for p in pts), 0.25 * sum(p[1] for p in pts))))
        elems.append(ids)

    coin = {}
    for j in range(n_r):
        for i in range(n_theta):
            if mirror and 2 * i >= n_theta:
                ac = not coin[(n_theta - 1 - i, j)]      # the mirror of A-C is B-D
            else:
                ac = bool(rng.random() < 0.5)
            coin[(i, j)] = ac
            ks = {(a, b): (24 * (i + a), 24 * (j + b)) for a in (0, 1) for b in (0, 1)}
            ps = {ab: corner(i + ab[0], j + ab[1]) for ab in ks}
            A, B, C, Dd = (0, 0), (1, 0), (1, 1), (0, 1)
            tris = [(A, B, C), (A, C, Dd)] if ac else [(A, B, Dd), (B, C, Dd)]
            for (p, qq, r) in tris:
                kp, kq, kr = ks[p], ks[qq], ks[r]
                pp, pq, pr = ps[p], ps[qq], ps[r]
                kg = ((kp[0] + kq[0] + kr[0]) // 3, (kp[1] + kq[1] + kr[1]) // 3)
                pg = ((pp[0] + pq[0] + pr[0]) / 3.0, (pp[1] + pq[1] + pr[1]) / 3.0)
                kpq, kqr, krp = mid(kp, kq), mid(kq, kr), mid(kr, kp)
                ppq, pqr, prp = pmid(pp, pq), pmid(pq, pr), pmid(pr, pp)
                add_quad([kp, kpq, kg, krp], [pp, ppq, pg, prp])
                add_quad([kq, kqr, kg, kpq], [pq, pqr, pg, ppq])
                add_quad([kr, krp, kg, kqr], [pr, prp, pg, pqr])
    P = np.array(pos, dtype=np.float64)
    if quarter_turn:
        P = np.stack([2.0 * center[0] - (P[:, 1] - center[1]) - center[0],
                      center[1] + (P[:, 0] - center[0])], axis=1)
    E = np.array(elems, dtype=np.int64)
    keys = np.empty((len(pos), 2), dtype=np.int64)
    for k, v in key_to_id.items():
        keys[v] = k
    # Morton renumbering over a uniform quantisation of the coordinates
    lo = P.min(axis=0)
    span = float((P.max(axis=0) - lo).max())
    qx = np.floor((P[:, 0] - lo[0]) / span * 65535.0).astype(np.int64)
    qy = np.floor((P[:, 1] - lo[1]) / span * 65535.0).astype(np.int64)
    order = np.argsort(_morton(qx, qy), kind="stable")
    new_id = np.empty_like(order)
    new_id[order] = np.arange(order.size)
    P, keys = P[order], keys[order]
    E = new_id[E]
    E = E[np.argsort(E[:, 8], kind="stable")]
    # wall nodes clockwise (theta key descending), far-field nodes
    on_wall = np.flatnonzero(keys[:, 1] == 0)
    wall = on_wall[np.argsort(-keys[on_wall, 0], kind="stable")]
    far = np.flatnonzero(keys[:, 1] == 24 * n_r)
    return UnstructuredMesh(P[:, 0].copy(), P[:, 1].copy(), E.astype(np.int32),
                            np.zeros((E.shape[0], 9, 2), dtype=np.int8), (0.0, 0.0),
                            info={"kind": "cylinder_q9", "n_theta": n_theta, "n_r": n_r, "D": D,
                                  "far_D": far_D, "seed": seed, "center": tuple(center),
                                  "mirror": mirror, "quarter_turn": quarter_turn},
                            wall_nodes=wall.astype(np.int32), far_nodes=far.astype(np.int32))


def q9_cylinder_case(n_theta: int = 32, D: float = 40.0, far_D: float = 6.0, seed: int = 1,
                     Ma: float = 0.2, Re: float = 100.0, T0: float = 1.0 / 3.0,
                     gamma: float = 1.4, Pr: float = 0.71, storage: int = 0,
                     mirror: bool = False, heave_D: float = 0.0, heave_St: float = 0.2):
    """Flow past a cylinder on the unstructured mesh of `cylinder_q9_mesh`:
    free stream along +x at Mach Ma, Re = rho U D / mu, started from
    potential flow times tanh((r - R) / delta) (delta = D / 8), uniform
    density and temperature; dt = (smallest patch reach) / (3 sqrt 2).
    Returns (mesh, fluid, body, (rho, ux, uy, T)); the body is fixed
    (elastic axis at the centre), or with heave_D > 0 in prescribed heave
    h = heave_D D sin(2 pi f t), f = heave_St U / D, rigid out to R + D/4 and
    blended out to R + 2D."""
    from .configs import DOF_FIXED, DOF_PRESCRIBED, BodyParams, FluidParams, sound_speed
    mesh = cylinder_q9_mesh(n_theta, D, far_D, seed=seed, mirror=mirror)
    U = Ma * sound_speed(gamma, T0)
    mu = 1.0 * U * D / Re
    dt = smallest_patch_reach(mesh) / (3.0 * np.sqrt(2.0))
    fluid = FluidParams(gamma=gamma, Pr=Pr, mu=mu, rho_inf=1.0, T_inf=T0, u_inf=(U, 0.0), dt=dt,
                        storage=storage)
    R = 0.5 * D
    if heave_D > 0.0:
        body = BodyParams(dof=DOF_PRESCRIBED, center=(0.0, 0.0), ea=(0.0, 0.0),
                          r_rigid=R + 0.25 * D, r_blend=R + 2.0 * D, heave_amp=heave_D * D,
                          heave_freq=heave_St * U / D)
    else:
        body = BodyParams(dof=DOF_FIXED, center=(0.0, 0.0), ea=(0.0, 0.0), r_rigid=R, r_blend=D)
    r = np.hypot(mesh.X, mesh.Y)
    c, s = mesh.X / r, mesh.Y / r
    a = (R / r) ** 2
    layer = np.tanh(np.maximum(r - R, 0.0) / (D / 8.0))
    ur = U * (1.0 - a) * c
    ut = -U * (1.0 + a) * s
    ux = (ur * c - ut * s) * layer
    uy = (ur * s + ut * c) * layer
    N = mesh.n_nodes
    return mesh, fluid, body, (np.ones(N), ux, uy, np.full(N, T0))


def q9_heave_case(n_theta: int = 32, D: float = 40.0, far_D: float = 6.0, seed: int = 1,
                  amp_D: float = 0.02, Ma_body: float = 0.05, T0: float = 1.0 / 3.0,
                  nu: float = 0.02, gamma: float = 1.4, Pr: float = 0.71, storage: int = 0,
                  dof: int = 0, mstar: float = 2.0, ustar: float = 5.0,
                  symmetric: bool = False, pitch_deg: float = 0.0, ea_D: float = 0.0,
                  distance_blend: bool = False):
    """A cylinder on the unstructured mesh of `cylinder_q9_mesh` in gas at
    rest, moving along y: prescribed heave h = A sin(w t) (dof 0; A = amp_D D,
    peak speed Ma_body times the speed of sound), or released at h0 = A with
    that peak speed on a spring (dof 1, mass ratio mstar, reduced velocity
    ustar against the same speed; the initial speed makes the fluid's load
    large against the rounding of single-precision populations, which a body
    released from rest feels only at that level in the first steps).
    pitch_deg > 0 (dof 0): also a prescribed pitch alpha = pitch_deg sin(w_a t)
    about the elastic axis (ea_D D, 0), the wall's peak pitching speed again
    Ma_body times the speed of sound.  Blending: rigid out to R + D/4 from the
    centre, blended out to R + 2D; distance_blend: the same distances measured
    from the wall polygon (D/4 and 2D).
    symmetric: the mesh is its own mirror image about the y axis (the line of
    the motion).
    dt = (smallest patch reach) / (3 sqrt 2).  Returns (mesh, fluid, body,
    (rho, ux, uy, T))."""
    from .configs import BodyParams, FluidParams, sound_speed
    mesh = cylinder_q9_mesh(n_theta, D, far_D, seed=seed, mirror=symmetric, quarter_turn=symmetric)
    R = 0.5 * D
    c = sound_speed(gamma, T0)
    A = amp_D * D
    w = Ma_body * c / A
    dt = smallest_patch_reach(mesh) / (3.0 * np.sqrt(2.0))
    fluid = FluidParams(gamma=gamma, Pr=Pr, mu=nu, rho_inf=1.0, T_inf=T0, u_inf=(0.0, 0.0), dt=dt,
                        storage=storage)
    m = mstar * np.pi * R * R
    U = Ma_body * c
    k_h = m * (2.0 * np.pi * U / (ustar * D)) ** 2
    a_amp = np.radians(pitch_deg) if dof == 0 else 0.0
    w_a = U / (a_amp * (R + abs(ea_D) * D)) if a_amp > 0 else 0.0
    r0 = 0.0 if distance_blend else R
    body = BodyParams(dof=dof, m=m, k_h=k_h, center=(0.0, 0.0), ea=(ea_D * D, 0.0),
                      r_rigid=r0 + 0.25 * D, r_blend=r0 + 2.0 * D, blend_mode=1 if distance_blend else 0,
                      heave_amp=A if dof == 0 else 0.0, heave_freq=w / (2.0 * np.pi) if dof == 0 else 0.0,
                      pitch_amp=a_amp, pitch_freq=w_a / (2.0 * np.pi),
                      h0=A if dof == 1 else 0.0, hd0=U if dof == 1 else 0.0)
    N = mesh.n_nodes
    return mesh, fluid, body, (np.ones(N), np.zeros(N), np.zeros(N), np.full(N, T0))


def q9_comoving_case(n_theta: int = 16, D: float = 20.0, far_D: float = 4.0, seed: int = 1,
                     Ma: float = 0.1, T0: float = 1.0 / 3.0, nu: float = 0.02, gamma: float = 1.4,
                     Pr: float = 0.71, storage: int = 0):
    """A cylinder carried along y by gas in uniform motion at Mach Ma: the
    body on a spring-free heave equation with a mass far above the gas's
    (1e30), started at the gas velocity, so that it keeps that velocity; the
    mesh blends rigid out to R + D/4 and back to rest at R + 1.2 D (inside
    the outer boundary).  Exactly, nothing changes but the body's position.
    Returns (mesh, fluid, body, (rho, ux, uy, T))."""
    from .configs import DOF_HEAVE, BodyParams, FluidParams, sound_speed
    mesh = cylinder_q9_mesh(n_theta, D, far_D, seed=seed)
    R = 0.5 * D
    U = Ma * sound_speed(gamma, T0)
    dt = smallest_patch_reach(mesh) / (3.0 * np.sqrt(2.0))
    fluid = FluidParams(gamma=gamma, Pr=Pr, mu=nu, rho_inf=1.0, T_inf=T0, u_inf=(0.0, U), dt=dt,
                        storage=storage)
    body = BodyParams(dof=DOF_HEAVE, m=1e30, k_h=0.0, center=(0.0, 0.0), ea=(0.0, 0.0),
                      r_rigid=R + 0.25 * D, r_blend=R + 1.2 * D, hd0=U)
    N = mesh.n_nodes
    return mesh, fluid, body, (np.ones(N), np.zeros(N), np.full(N, U), np.full(N, T0))
