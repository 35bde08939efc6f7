"""Departure points on strongly skewed and twisted cells (Sec. II.B: the
departure point X - dt c^ located in the computational coordinates of the
first-order element holding it).

The oracle solves the bilinear map of each candidate cell by Newton's method.
These tests evaluate the forward map instead: the bilinear interpolation of
the cell's four corner nodes at the returned offsets must give the departure
point itself, on a periodic mesh whose j lines lean 60 degrees from the normal
and whose cells are twisted by up to 0.15 of a cell (the range where the
kernel's fixed point needs more than its three unconditional rounds), and on
the twin O-grid, whose junction cells are the most distorted of the
structured meshes here.
"""

import numpy as np
import pytest

import synth
from oracle import lattice as L
from oracle import mesh as M
from oracle import stream as S


def forward_point(grid, X, Y, a, b):
    """X(xi + (a, b)) - X(xi) by bilinear interpolation in the cell holding
    (a, b): lower-left corner offset -1 or 0 in each index."""
    i0 = np.where(a < 0.0, -1, 0)
    j0 = np.where(b < 0.0, -1, 0)
    s = a - i0
    t = b - j0
    px = np.zeros(X.shape)
    py = np.zeros(X.shape)
    for di0 in (-1, 0):
        for dj0 in (-1, 0):
            sel = (i0 == di0) & (j0 == dj0)
            if not sel.any():
                continue
            for ci, cj, w in ((0, 0, (1 - s) * (1 - t)), (1, 0, s * (1 - t)),
                              (0, 1, (1 - s) * t), (1, 1, s * t)):
                cx, cy = grid.neighbour_pos(X, Y, di0 + ci, dj0 + cj)
                px = np.where(sel, px + w * (cx - X), px)
                py = np.where(sel, py + w * (cy - Y), py)
    return px, py


def check_directions(grid, X, Y, dt, wall_row=False):
    # far-field nodes take the boundary condition, not a departure point
    active = ~S.boundary_nodes(grid)
    worst = 0.0
    for i in range(9):
        chx = np.where(active, float(L.CX[i]), 0.0)
        chy = np.where(active, float(L.CY[i]), 0.0)
        a, b, miss = S.departure_offsets(grid, X, Y, chx, chy, dt, wall_row=wall_row)
        ok = ~miss & active
        assert np.all(np.isfinite(a[ok])) and np.all(np.abs(a[ok]) <= 1 + 1e-12)
        assert np.all(np.abs(b[ok]) <= 1 + 1e-12)
        px, py = forward_point(grid, X, Y, np.where(ok, a, 0.0), np.where(ok, b, 0.0))
        err = np.hypot(px + dt * L.CX[i], py + dt * L.CY[i])[ok]
        worst = max(worst, float(np.max(err)))
    return worst


def test_departure_points_on_skewed_twisted_cells_map_back():
    mesh = synth.skewed_twisted_mesh()
    grid = M.Grid.from_mesh(mesh)
    # the cells really are that distorted: twist of the x coordinate per cell
    X = mesh.X
    tw = X[1:, 1:] - X[1:, :-1] - X[:-1, 1:] + X[:-1, :-1]
    assert np.max(np.abs(tw)) > 0.14
    assert check_directions(grid, mesh.X, mesh.Y, 0.2) < 1e-12


def test_departure_points_near_the_twin_junction_map_back():
    c = synth.small_tandem_case()
    grid = M.Grid.from_mesh(c.mesh)
    scale = float(np.max(np.hypot(np.diff(c.mesh.X, axis=1), np.diff(c.mesh.Y, axis=1))))
    assert check_directions(grid, c.mesh.X, c.mesh.Y, c.fluid.dt, wall_row=True) < 1e-12 * scale


@pytest.mark.parametrize("wrong", ["transposed", "sign"])
def test_forward_check_detects_a_wrong_solve(wrong):
    """The forward evaluation catches offsets with a plausible mistake."""
    mesh = synth.skewed_twisted_mesh()
    grid = M.Grid.from_mesh(mesh)
    dt = 0.2
    chx = np.full(mesh.X.shape, 1.0)
    chy = np.full(mesh.X.shape, 1.0)
    a, b, _ = S.departure_offsets(grid, mesh.X, mesh.Y, chx, chy, dt)
    a2, b2 = (b, a) if wrong == "transposed" else (-a, b)
    px, py = forward_point(grid, mesh.X, mesh.Y, a2, b2)
    assert np.max(np.hypot(px + dt, py + dt)) > 1e-2
