"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds input generators only: mesh node coordinates, initial
macroscopic fields and physical parameters expressed in lattice units.  It
contains none of the lattice Boltzmann arithmetic (no equilibria, no
streaming, no boundary rules), so that the HIP library and the FP64 oracle
can be fed identical inputs without sharing any of the method's code.
"""

from .meshes import (  # noqa: F401
    MeshSpec,
    periodic_sine_mesh,
    cartesian_mesh,
    ogrid_mesh,
    cgrid_mesh,
    twin_mesh,
    skewed_twisted_mesh,
    geometric_ratio,
)
from .configs import (  # noqa: F401
    FluidParams,
    BodyParams,
    acoustic_pulse_case,
    cylinder_viv_case,
    large_heave_case,
    batched_sweep_cases,
    gaussian_pulse_fields,
    airfoil_flutter_case,
    small_airfoil_case,
    tandem_cylinders_case,
    small_tandem_case,
)
