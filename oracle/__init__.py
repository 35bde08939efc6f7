"""Plain FP64 CPU oracle of the two-population compressible lattice Boltzmann
FSI step (Bhadauria, Dorschner & Karlin, arXiv 2107.01370).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` use it.  It shares no code with the
HIP library (its only common dependency is the ``synth`` input generators,
which hold none of the method's arithmetic).

The oracle is deliberately slow and literal: NumPy float64, vectorised over
mesh nodes, with explicit Python loops over the nine D2Q9 velocities and over
stencil taps.  Every function cites the passage of the paper it follows.
Where the paper is silent or garbled, the reading taken is stated in the
docstring.

Modules
-------
lattice   D2Q9 velocities, weights, moments, equilibria, correction terms,
          collision (Sec. II.C).
mesh      FE derivatives on the structured mesh, blending-function mesh motion
          (Sec. II.A, II.B, II.D).
stream    ALE departure points, bilinear inverse map, biquadratic Lagrange
          interpolation (Sec. II.A-B).
boundary  Grad wall boundary condition and far-field equilibria (Sec. III.A).
forces    surface force and moment (Sec. III).
body      1DOF / 2DOF rigid-body ODEs and RK4 (Sec. IV).
solver    the staggered fluid-structure step (Sec. III).
"""

from . import lattice, mesh, stream, boundary, forces, body, solver  # noqa: F401
