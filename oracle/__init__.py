"""FP64 CPU oracle for the Hermite-matrix MRT lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  This package is the parity authority for the HIP
path: a plain, slow, vectorised NumPy implementation written directly from the
paper (Shi, Yuan & Chai, "A unified MRT-LB framework for Navier-Stokes and
nonlinear convection-diffusion equations and beyond", arXiv 2512.16230).
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library and the
library never imports it.

Modules
-------
lattice  velocity sets, weight solvers, Hermite rows (Sec. V, App. C, App. D)
model    one time step of eq. (2-3) with the Hermite collision of
         eq. (H-MRT-LB-1); NSE (Sec. III/IV) and NCDE (App. A) moments
naive    brute-force formulation (explicit b x b collision matrix in
         velocity space, per-population loop streaming) used to pin ``model``
"""

from . import lattice, model, naive  # noqa: F401
