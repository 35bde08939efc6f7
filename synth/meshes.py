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
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TOPO_PERIODIC2 = 0
TOPO_OGRID = 1
TOPO_CGRID = 2


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
