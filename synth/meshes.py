"""Structured curvilinear meshes in lattice units (node coordinates only).

Index convention used everywhere in this repository: node (i, j) with i the
fastest (periodic / azimuthal) index and j the slow (wall-normal) index.
Arrays are shaped [nj, ni].  The computational coordinates of node (i, j) are
the continuous indices xi = (i, j).

Topologies
----------
``TOPO_PERIODIC2`` (0)
    periodic in i and in j.  Crossing the seam in i adds ``shift_i`` to the
    coordinates, crossing it in j adds ``shift_j``.
``TOPO_OGRID`` (1)
    periodic in i without a coordinate shift; row j = 0 is a solid wall and row
    j = nj - 1 is the far-field boundary.  Nodes run clockwise in i so that
    det(d(x, y)/d(i, j)) > 0 with j pointing into the fluid.
``TOPO_CGRID`` (2)
    C-grid around an airfoil with a wake cut: i runs from the lower end of the
    cut (downstream exit), along the lower side of the cut to the trailing
    edge, round the airfoil (lower surface, leading edge, upper surface) back
    to the trailing edge and along the upper side of the cut to the exit.
    ``n_wake`` nodes lie on each side of the cut; the trailing edge appears
    twice (i = n_wake and i = ni - 1 - n_wake) and every cut node (i, 0)
    coincides with (ni - 1 - i, 0).  Row j = 0 between the trailing-edge
    copies is the wall; row j = nj - 1 and columns i = 0, ni - 1 are far field.
``TOPO_TWIN`` (3)
    O-grid around two bodies joined by a slit (a cut of zero thickness):
    periodic in i, row j = nj - 1 far field.  Row 0 runs round the first
    body (columns 0 .. nA, both ends the same junction point), along one side
    of the slit (``n_wake`` cells), round the second body (``n_wall2`` cells,
    both ends the other junction point) and back along the other side of the
    slit, with ni = nA + 2 n_wake + n_wall2.  Across the slit node (i, -m) is
    node ((nA - i) mod ni, m).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TOPO_PERIODIC2 = 0
TOPO_OGRID = 1
TOPO_CGRID = 2
TOPO_TWIN = 3


@dataclass
class MeshSpec:
    ni: int
    nj: int
    topo: int
    X: np.ndarray  # [nj, ni] float64, undeformed x coordinate
    Y: np.ndarray  # [nj, ni] float64, undeformed y coordinate
    shift_i: tuple = (0.0, 0.0)
    shift_j: tuple = (0.0, 0.0)
    info: dict = field(default_factory=dict)
    n_wake: int = 0            # C-grid: nodes on each side of the wake cut; twin O-grid: slit cells
    n_wall2: int = 0           # twin O-grid: wall cells round the second body

    @property
    def n_nodes(self) -> int:
        return self.ni * self.nj

    def interleaved(self) -> np.ndarray:
        """Coordinates as one contiguous float64 array [nj][ni][2]."""
        out = np.empty((self.nj, self.ni, 2), dtype=np.float64)
        out[..., 0] = self.X
        out[..., 1] = self.Y
        return out


def cartesian_mesh(ni: int, nj: int, spacing: float = 1.0) -> MeshSpec:
    """Undeformed doubly periodic unit grid (period ni*spacing x nj*spacing)."""
    jj, ii = np.meshgrid(np.arange(nj, dtype=np.float64),
                         np.arange(ni, dtype=np.float64), indexing="ij")
    return MeshSpec(ni, nj, TOPO_PERIODIC2, ii * spacing, jj * spacing,
                    shift_i=(ni * spacing, 0.0), shift_j=(0.0, nj * spacing),
                    info={"kind": "cartesian", "spacing": spacing})


def periodic_sine_mesh(n: int = 64, amp: float = 0.05, ni: int | None = None,
                       nj: int | None = None) -> MeshSpec:
    """Unit Cartesian grid with x += amp sin(2 pi y / nj), y += amp sin(2 pi x / ni).

    With the defaults this is the static 64 x 64 periodic curvilinear mesh of
    the acoustic-pulse workload.
    """
    ni = n if ni is None else ni
    nj = n if nj is None else nj
    jj, ii = np.meshgrid(np.arange(nj, dtype=np.float64),
                         np.arange(ni, dtype=np.float64), indexing="ij")
    X = ii + amp * np.sin(2.0 * np.pi * jj / nj)
    Y = jj + amp * np.sin(2.0 * np.pi * ii / ni)
    return MeshSpec(ni, nj, TOPO_PERIODIC2, X, Y,
                    shift_i=(float(ni), 0.0), shift_j=(0.0, float(nj)),
                    info={"kind": "periodic_sine", "amp": amp})


def skewed_twisted_mesh(n: int = 32, skew_deg: float = 60.0, twist: float = 0.3,
                        wavelength: int = 8) -> MeshSpec:
    """Doubly periodic mesh of strongly skewed, twisted cells.

    x = i + tan(skew) j + twist sin(k i) sin(k j), y = j, with k = 2 pi /
    wavelength: the j lines lean by ``skew_deg`` from the normal to the i
    lines, and each cell is twisted (its fourth corner leaves the
    parallelogram of the other three) by up to 4 twist sin^2(k / 2) cells
    (0.15 with the defaults, on the nodes); dx/di stays between 1 - twist k
    and 1 + twist k.
    """
    if n % wavelength:
        raise ValueError("the wavelength must divide n")
    sh = float(np.tan(np.radians(skew_deg)))
    k = 2.0 * np.pi / wavelength
    jj, ii = np.meshgrid(np.arange(n, dtype=np.float64),
                         np.arange(n, dtype=np.float64), indexing="ij")
    X = ii + sh * jj + twist * np.sin(k * ii) * np.sin(k * jj)
    Y = jj.copy()
    return MeshSpec(n, n, TOPO_PERIODIC2, X, Y,
                    shift_i=(float(n), 0.0), shift_j=(sh * n, float(n)),
                    info={"kind": "skewed_twisted", "skew_deg": skew_deg, "twist": twist,
                          "wavelength": wavelength})


def geometric_ratio(n_cells: int, first: float, span: float) -> float:
    """Ratio q with first * (q**n_cells - 1) / (q - 1) == span (bisection)."""
    if abs(first * n_cells - span) < 1e-12 * span:
        return 1.0
    lo, hi = 1.0 + 1e-15, 1.0 + min(1.0, 700.0 / n_cells)   # q**n_cells stays finite
    if first * n_cells > span:
        lo, hi = 1e-6, 1.0 - 1e-15

    def total(q):
        return first * (q ** n_cells - 1.0) / (q - 1.0)

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (total(mid) - span) * (total(lo) - span) > 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def ogrid_mesh(n_r: int, n_theta: int, diameter: float, first_cell: float,
               r_far: float, center=(0.0, 0.0)) -> MeshSpec:
    """O-grid around a circle of the given diameter.

    Radial node j sits at r_j = R + first_cell * (q**j - 1) / (q - 1), with the
    geometric ratio q chosen so that r_{n_r-1} = r_far.  Azimuthal node i sits
    at theta_i = -2 pi i / n_theta (clockwise, so that j points into the fluid
    with a positive Jacobian).
    """
    R = 0.5 * diameter
    q = geometric_ratio(n_r - 1, first_cell, r_far - R)
    j = np.arange(n_r, dtype=np.float64)
    if q == 1.0:
        r = R + first_cell * j
    else:
        r = R + first_cell * (q ** j - 1.0) / (q - 1.0)
    r[-1] = r_far
    theta = -2.0 * np.pi * np.arange(n_theta, dtype=np.float64) / n_theta
    X = center[0] + r[:, None] * np.cos(theta)[None, :]
    Y = center[1] + r[:, None] * np.sin(theta)[None, :]
    return MeshSpec(n_theta, n_r, TOPO_OGRID, X, Y,
                    info={"kind": "ogrid", "diameter": diameter,
                          "first_cell": first_cell, "r_far": r_far, "ratio": q,
                          "center": tuple(center)})


def naca_thickness(x: np.ndarray, chord: float, t: float) -> np.ndarray:
    """Half-thickness of a symmetric NACA 4-digit section with a closed
    trailing edge (last coefficient -0.1036 instead of -0.1015)."""
    u = np.clip(x / chord, 0.0, 1.0)
    return 5.0 * t * chord * (0.2969 * np.sqrt(u) - 0.1260 * u - 0.3516 * u ** 2
                              + 0.2843 * u ** 3 - 0.1036 * u ** 4)


def _airfoil_nodes(n_af: int, chord: float, t: float, cluster: float):
    """Wall nodes from the lower trailing edge round the leading edge to the
    upper trailing edge (both trailing-edge copies included), spaced in arc
    length with density 1 - cluster cos(4 pi u): finest at the trailing and
    leading edges, coarsest at mid-chord."""
    # dense parametrisation: x = c (1 + cos(2 pi s)) / 2, lower surface for s < 1/2
    s = np.linspace(0.0, 1.0, 200001)
    x = 0.5 * chord * (1.0 + np.cos(2.0 * np.pi * s))
    y = np.where(s < 0.5, -1.0, 1.0) * naca_thickness(x, chord, t)
    seg = np.hypot(np.diff(x), np.diff(y))
    S = np.concatenate([[0.0], np.cumsum(seg)])
    u = np.arange(n_af, dtype=np.float64) / (n_af - 1)
    phi = u - cluster * np.sin(4.0 * np.pi * u) / (4.0 * np.pi)
    target = phi * S[-1]
    sk = np.interp(target, S, s)
    xk = 0.5 * chord * (1.0 + np.cos(2.0 * np.pi * sk))
    yk = np.where(sk < 0.5, -1.0, 1.0) * naca_thickness(xk, chord, t)
    xk[0] = xk[-1] = chord
    yk[0] = yk[-1] = 0.0
    # exact mirror symmetry about the chord line
    half = n_af // 2
    xk[n_af - half:] = xk[:half][::-1]
    yk[n_af - half:] = -yk[:half][::-1]
    return xk, yk


def cgrid_mesh(n_wake: int, n_af: int, nj: int, chord: float, first_cell: float,
               far_chords: float, t: float = 0.12, cluster: float = 0.6,
               origin=(0.0, 0.0)) -> MeshSpec:
    """C-grid around a NACA 00xx airfoil (leading edge at ``origin``, chord
    along +x) from the parabolic map z = zeta^2 + x_o, with x_o half the
    leading-edge radius so that the map's branch point lies inside the nose.

    In the zeta = xi + i eta half plane the wake cut is eta = 0 and the
    airfoil a graph eta_w(xi); column i is the line xi = xi_i, row j sits at
    eta_w + (eta_max - eta_w) * (geometric fraction) with the first step
    chosen so that the first physical cell is about ``first_cell`` long.  The
    outer parabola eta = eta_max passes far_chords * chord upstream of the
    leading edge and the exit columns far_chords * chord downstream of the
    trailing edge; every far-field point is at least that far from the
    leading edge.  The mesh is mirror-symmetric about the chord line.
    """
    if n_af % 2 or n_wake < 2:
        raise ValueError("n_af must be even and n_wake >= 2")
    ni = 2 * n_wake + n_af
    x_o = 0.5 * 1.1019 * t * t * chord
    xa, ya = _airfoil_nodes(n_af, chord, t, cluster)
    # wake cut: from the trailing edge to the exit, geometric in x starting
    # with the trailing-edge spacing of the airfoil nodes
    te_step = float(np.hypot(xa[1] - xa[0], ya[1] - ya[0]))
    q = geometric_ratio(n_wake, te_step, far_chords * chord)
    k = np.arange(1, n_wake + 1, dtype=np.float64)
    xw = chord + te_step * (q ** k - 1.0) / (q - 1.0)
    xw[-1] = chord * (1.0 + far_chords)
    # wall / cut points in the zeta plane (branch with Im zeta >= 0)
    zw = (xa - x_o) + 1j * ya
    ang = np.mod(np.angle(zw), 2.0 * np.pi)
    zeta_af = np.sqrt(np.abs(zw)) * np.exp(0.5j * ang)
    zeta_af[0] = -np.sqrt(chord - x_o)
    zeta_af[-1] = np.sqrt(chord - x_o)
    xi_w = np.sqrt(xw - x_o)
    xi = np.concatenate([-xi_w[::-1], zeta_af.real, xi_w[::-1][::-1]])
    eta_w = np.concatenate([np.zeros(n_wake), np.maximum(zeta_af.imag, 0.0), np.zeros(n_wake)])
    eta_max = np.sqrt(far_chords * chord + x_o)
    # per-column geometric distribution in eta; physical step ~ 2 |zeta| d eta
    X = np.empty((nj, ni))
    Y = np.empty((nj, ni))
    jj = np.arange(nj, dtype=np.float64)
    for i in range(ni):
        zmag = max(abs(complex(xi[i], eta_w[i])), 1e-12)
        d_eta = first_cell / (2.0 * zmag)
        span = eta_max - eta_w[i]
        qi = geometric_ratio(nj - 1, d_eta, span)
        frac = jj if qi == 1.0 else (qi ** jj - 1.0) / (qi - 1.0)
        eta = eta_w[i] + d_eta * frac
        eta[-1] = eta_max
        z = (xi[i] + 1j * eta) ** 2 + x_o
        X[:, i] = z.real
        Y[:, i] = z.imag
    # wall row exactly on the section; the upper half is the exact mirror image
    # of the lower half (so the cut rows are exactly duplicated)
    X[0, n_wake:n_wake + n_af] = xa
    Y[0, n_wake:n_wake + n_af] = ya
    lo = np.arange(ni // 2)
    X[:, ni - 1 - lo] = X[:, lo]
    Y[:, ni - 1 - lo] = -Y[:, lo]
    Y[0, :n_wake + 1] = 0.0
    Y[0, ni - 1 - n_wake:] = 0.0
    X += origin[0]
    Y += origin[1]
    return MeshSpec(ni, nj, TOPO_CGRID, X, Y, n_wake=n_wake,
                    info={"kind": "cgrid", "n_wake": n_wake, "chord": chord,
                          "thickness": t, "first_cell": first_cell,
                          "far_chords": far_chords, "x_o": x_o, "wake_ratio": q,
                          "origin": tuple(origin)})


def _bipolar(w, a):
    """Bipolar coordinates w = sigma + i tau -> z = a (1 + e^{iw}) / (1 - e^{iw})
    (x = a sinh tau / (cosh tau - cos sigma), y = a sin sigma / (cosh tau -
    cos sigma)): tau = +-tau_0 are circles round the foci (+-a, 0), sigma = +-pi
    the segment between them, and w = 0 is the point at infinity."""
    e = np.exp(1j * w)
    return a * (1.0 + e) / (1.0 - e)


def twin_mesh(n_wall: int, n_slit: int, nj: int, diameter: float, spacing: float,
              first_cell: float, far_diameters: float, samples: int = 6000) -> MeshSpec:
    """Twin O-grid round two circles of the given diameter whose centres lie
    ``spacing`` apart on the x axis (at -+ spacing / 2), joined by a slit
    along the x axis between them.

    Bipolar coordinates with the circles as tau = -+tau_0 map the rectangle
    |sigma| <= pi, |tau| <= tau_0 conformally onto the plane outside the two
    circles and the slit (the edges sigma = +-pi are the slit's two sides and
    the rectangle's corners the two junctions of each side with the circles);
    its centre is the point at infinity.  Row j = 0 holds ``n_wall`` equal
    arcs on each circle and ``n_slit`` equal steps along the slit; column i
    follows the straight line from its wall point w_b to the centre,
    w = w_b (eps / |w_b|)^lambda with |w| = eps the far boundary (a near-circle
    of radius far_diameters * diameter), and its nodes are placed by arc
    length, geometric from ``first_cell``.  Straight lines to the centre of a
    rectangle do not cross, so no cell folds; cells next to the junctions are
    skewed (the fluid angle there is 90 degrees).  The mesh is exactly
    symmetric about both axes (columns i and (nA - i) mod ni mirror in y,
    i and (nA + n_slit + n_wall - i) mod ni in x).
    """
    if n_wall % 2 or n_wall < 8 or n_slit < 2:
        raise ValueError("n_wall must be even and >= 8, n_slit >= 2")
    R = 0.5 * diameter
    d = 0.5 * spacing
    if not d > R:
        raise ValueError("the circles overlap")
    a = float(np.sqrt(d * d - R * R))
    tau0 = float(np.arccosh(d / R))
    nA = nB = n_wall
    s = n_slit
    ni = nA + 2 * s + nB
    zb = np.empty(ni, dtype=complex)
    wb = np.empty(ni, dtype=complex)

    def w_of(z, tau):
        return np.angle((z - a) / (z + a)) + 1j * tau

    th = -2.0 * np.pi * np.arange(nA + 1) / nA           # clockwise from the junction
    zA = -d + R * np.cos(th) + 1j * R * np.sin(th)
    zb[:nA + 1] = zA
    wb[:nA + 1] = w_of(zA, -tau0)
    xs = -(d - R) + (spacing - diameter) * np.arange(s + 1) / s
    zb[nA:nA + s + 1] = xs
    wb[nA:nA + s + 1] = np.pi + 2j * np.arctanh(xs / a)
    th = np.pi - 2.0 * np.pi * np.arange(nB + 1) / nB
    zB = d + R * np.cos(th) + 1j * R * np.sin(th)
    zb[nA + s:nA + s + nB + 1] = zB
    wb[nA + s:nA + s + nB + 1] = w_of(zB, tau0)
    low = np.arange(nA + s + nB, ni)
    xl = xs[::-1][:-1]
    zb[low] = xl
    wb[low] = -np.pi + 2j * np.arctanh(xl / a)
    for i, wc in ((0, -np.pi - 1j * tau0), (nA, np.pi - 1j * tau0),
                  (nA + s, np.pi + 1j * tau0), (nA + s + nB, -np.pi + 1j * tau0)):
        wb[i] = wc
    # points on the axes: the far sides of the circles and the slit's middle
    for i, x in ((nA // 2, -d - R), (nA + s + nB // 2, d + R)):
        zb[i] = x
        wb[i] = 1j * wb[i].imag
    if s % 2 == 0:
        for i in (nA + s // 2, nA + s + nB + s // 2):
            zb[i] = 0.0
            wb[i] = wb[i].real
    eps = 2.0 * a / (far_diameters * diameter)
    lam = (np.arange(samples + 1) / samples) ** 2.5
    shrink = eps / np.abs(wb)
    W = wb[:, None] * shrink[:, None] ** lam[None, :]
    Z = _bipolar(W, a)
    Z[:, 0] = zb
    S = np.concatenate([np.zeros((ni, 1)), np.cumsum(np.abs(np.diff(Z, axis=1)), axis=1)], axis=1)
    X = np.empty((nj, ni))
    Y = np.empty((nj, ni))
    jj = np.arange(nj, dtype=np.float64)
    for i in range(ni):
        q = geometric_ratio(nj - 1, first_cell, S[i, -1])
        r = first_cell * jj if q == 1.0 else first_cell * (q ** jj - 1.0) / (q - 1.0)
        r[-1] = S[i, -1]
        li = np.interp(r, S[i], lam)
        z = _bipolar(wb[i] * shrink[i] ** li, a)
        z[0] = zb[i]
        X[:, i] = z.real
        Y[:, i] = z.imag
    # exact symmetries: mirror in y (source sigma > 0), then in x (source tau < 0)
    cols = np.arange(ni)
    my = (nA - cols) % ni
    up = wb.real > 0
    X[:, my[up]] = X[:, up]
    Y[:, my[up]] = -Y[:, up]
    Y[:, wb.real == 0] = 0.0
    mx = (nA + s + nB - cols) % ni
    left = wb.imag < 0
    X[:, mx[left]] = -X[:, left]
    Y[:, mx[left]] = Y[:, left]
    X[:, wb.imag == 0] = 0.0
    Y[0, nA:nA + s + 1] = 0.0
    Y[0, low] = 0.0
    Y[0, 0] = 0.0
    return MeshSpec(ni, nj, TOPO_TWIN, X, Y, n_wake=s, n_wall2=nB,
                    info={"kind": "twin", "diameter": diameter, "spacing": spacing,
                          "first_cell": first_cell, "far_diameters": far_diameters,
                          "n_wall": n_wall, "n_slit": s, "centers": ((-d, 0.0), (d, 0.0)),
                          "focus": a, "tau0": tau0})
