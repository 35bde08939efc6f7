"""MI355X (gfx950) implementation of the two-population compressible lattice
Boltzmann FSI step of arXiv 2107.01370.

The numerical work lives in the HIP library ``lib/libfsilbm.so`` behind the C
ABI ``include/fsilbm.h``; ``paper_2107_01370_amd.fsilbm`` is its Python
binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it has not been built.
"""

__all__ = ["fsilbm"]
