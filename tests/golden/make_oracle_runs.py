"""Writes the stored oracle results that the long GPU parity runs compare
against (the GPU tests read these files; nothing here touches the GPU).

Each run starts from the oracle's own float64 equilibria of the case's start
fields and steps the plain FP64 oracle (oracle/solver.py):

  force_protocol_cylinder_64x128.npz
      cylinder VIV on a 64 x 128 O-grid with the single-cylinder case's
      physics (Ma 0.2, Re 100, m* 10, U* 5, far field 30 D, blending to 10 D),
      D = 40 lattice units (first cell 0.025 D), released at h(0) = 0.01 D,
      2000 steps: the body history (n, F_x, F_y, M_EA, h, alpha) of every level
      and the final density and temperature fields.
  heave_cylinder_64x128_1000.npz
      the heaving-cylinder construction of the large workload (square wall
      cells, geometric stretching to 30 D, Ma 0.5, Re 1000, prescribed heave
      0.2 D at frequency 0.2 U / D) at 64 x 128 nodes with D = 50, 1000 steps:
      the body history and the density and temperature fields after 100 and
      after 1000 steps.
  cylinder_viv_256x512_200
      the single-cylinder workload at its own size (256 x 512 O-grid, first
      cell 0.005 D, far field 30 D, blending to 10 D; Ma 0.2, Re 100, m* 10,
      U* 5), 200 steps: the body history and the density and temperature of
      the rows listed in ROWS (wall, near-wall and every octave outward).

Usage: python tests/golden/make_oracle_runs.py [name ...]
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.solver import OracleSolver  # noqa: E402


def force_protocol_case():
    return synth.cylinder_viv_case(n_r=64, n_theta=128, D=40.0, first_cell_frac=0.025,
                                   r_far_D=30.0, blend_D=10.0, h0_frac=0.01, mstar=10.0,
                                   ustar=5.0, Ma=0.2, Re=100.0, steps=2000)


def heave_case():
    c = synth.large_heave_case(n_r=64, n_theta=128, D=50.0)
    c.steps = 1000
    return c


def cylinder_viv_256x512_case():
    c = synth.cylinder_viv_case()
    c.steps = 200
    return c


RUNS = {
    "force_protocol_cylinder_64x128": force_protocol_case,
    "heave_cylinder_64x128_1000": heave_case,
    "cylinder_viv_256x512_200": cylinder_viv_256x512_case,
}
# runs whose final fields are stored on these rows (radial index j) only
ROWS = {"cylinder_viv_256x512_200": (0, 1, 2, 4, 8, 16, 32, 64, 128, 192, 255)}
# intermediate levels whose fields are stored too
SNAPSHOTS = {"heave_cylinder_64x128_1000": (100,)}


def path_of(name: str) -> str:
    return os.path.join(HERE, name + ".npz")


def run(name: str, steps: int | None = None, snapshots=()):
    """The oracle run of `name` (all its steps, or the first `steps`); also
    the fields at the levels in `snapshots`."""
    c = RUNS[name]()
    n = c.steps if steps is None else steps
    ora = OracleSolver(c.mesh, c.fluid, c.bodies, c.rho, c.ux, c.uy, c.T)
    snaps = {}
    done = 0
    for m in sorted(k for k in snapshots if k < n):
        ora.run(m - done)
        done = m
        rho, ux, uy, E, T = ora.macroscopic()
        snaps[m] = (rho, T)
    ora.run(n - done)
    rho, ux, uy, E, T = ora.macroscopic()
    return c, np.array(ora.history, dtype=np.float64), rho, T, snaps


def main(names):
    for name in names:
        t0 = time.time()
        c, hist, rho, T, snaps = run(name, snapshots=SNAPSHOTS.get(name, ()))
        meta = {"case": name, "steps": c.steps, "nodes": c.mesh.ni * c.mesh.nj,
                "dt": c.fluid.dt, "snapshots": sorted(snaps),
                "info": {k: float(v) for k, v in c.info.items() if isinstance(v, (int, float))}}
        extra = {}
        if name in ROWS:
            rows = np.array(ROWS[name], dtype=np.int64)
            rho, T = rho[rows], T[rows]
            extra["rows"] = rows
        for m, (r, t) in snaps.items():
            extra[f"rho_{m}"] = r
            extra[f"T_{m}"] = t
        np.savez_compressed(path_of(name), history=hist, rho=rho, T=T,
                            meta=np.array(json.dumps(meta)), **extra)
        print(f"{name}: {c.steps} steps in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(RUNS))
