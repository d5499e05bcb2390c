"""Write the FP64 oracle references of the 256 x 256 rD2Q25 Taylor-Green
runs used by the mixed-precision accuracy test (tgv256_refs.npz).

Calls only oracle/ and the seeded input generators.  Workload: the
benchmark physics on a 256 x 256 periodic box (dx/dy = 1.5, Ma = 0.1,
tau_shear = 0.6, other rates 1.2), 1000 steps, with and without the
N(0, 1e-3^2) velocity perturbation.  Run from the repository root:

    python tests/golden/make_tgv256_references.py
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lattice as OL  # noqa: E402
from oracle import model as OM  # noqa: E402
from paper_2512_16230_amd import workloads as W  # noqa: E402

SHAPE = (256, 256)
STEPS = 1000


def run(sigma):
    wl = W.tgv_large(0, shape=SHAPE, steps=STEPS, sigma=sigma)
    card, r = wl.card, wl.rates
    lat = OL.make_lattice(card.kind, card.c, card.cs2, card.free)
    mdl = OM.Model(eq=wl.eq, s0=r.s0, s1=r.s1, s_shear=r.s_shear, s_bulk=r.s_bulk, s3=r.s3, s_h=r.s_h)
    st = OM.init_state(lat, mdl, wl.rho_or_phi, wl.u)
    t0 = time.time()
    st = OM.run(lat, mdl, st, STEPS)
    rho, u = OM.moments(lat, mdl, st)
    print("sigma %g: %d steps in %.0f s" % (sigma, STEPS, time.time() - t0), flush=True)
    return rho, u


def main():
    rho_n, u_n = run(1e-3)
    rho_c, u_c = run(0.0)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv256_refs.npz")
    np.savez_compressed(out, rho_noise=rho_n, u_noise=u_n, rho_clean=rho_c, u_clean=u_c,
                        steps=STEPS, shape=np.array(SHAPE))
    print("wrote", out)


if __name__ == "__main__":
    main()
