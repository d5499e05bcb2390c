"""MI355X-native Hermite-matrix MRT lattice Boltzmann (arXiv 2512.16230).

The compute path is the HIP library ``libmrtlb.so`` (sources in ``csrc/``,
C ABI in ``include/mrtlb.h``); ``_mrtlb`` is its ctypes binding.  There is
no CPU fallback: calls fail if the library is not built.
"""

from ._mrtlb import (  # noqa: F401
    Context, Lattice, MrtlbError, Solve, batch_step, footprint, lib, model_desc,
)
