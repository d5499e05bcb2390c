"""Shared helpers of the parity tests: build the oracle and the HIP solve
from the same workload parameters and compare them."""

import os

import numpy as np

from oracle import lattice as OL
from oracle import model as OM


def oracle_for(card, eq, rates, rho0=1.0, D0=0.0, D2=0.0, adv=(0.0, 0.0, 0.0), m30=True, gn_bt=(0.0, 0.0, 0.0),
               gn_dd=(0.0, 0.0, 0.0), src_q=0.0, src_k=0.0, three_level=False, mass_src=0.0, g_share=0.0,
               lambda1=1.0, lambda2=1.0, m2g_form=0):
    lat = OL.make_lattice(card.kind, card.c, card.cs2, card.free)
    mdl = OM.Model(eq=eq, rho0=rho0, s0=rates.s0, s1=rates.s1, s_shear=rates.s_shear, s_bulk=rates.s_bulk,
                   s3=rates.s3, s_h=rates.s_h, m30=m30, D0=D0, D2=D2, adv_u=tuple(adv), gn_bt=tuple(gn_bt),
                   gn_dd=tuple(gn_dd), src_q=src_q, src_k=src_k, three_level=three_level, mass_src=mass_src,
                   g_share=g_share, lambda1=lambda1, lambda2=lambda2, m2g_form=m2g_form)
    return lat, mdl


def hip_model(eq, rates, rho0=1.0, D0=0.0, D2=0.0, adv=(0.0, 0.0, 0.0), m30=True, u_bound=0.0, dev_bound=0.0,
              gn_bt=(0.0, 0.0, 0.0), gn_dd=(0.0, 0.0, 0.0), src_q=0.0, src_k=0.0, three_level=False,
              mass_src=0.0, g_share=0.0, lambda1=1.0, lambda2=1.0, m2g_form=0):
    from paper_2512_16230_amd import _mrtlb as H
    return H.model_desc(eq, rho0=rho0, s0=rates.s0, s1=rates.s1, s_shear=rates.s_shear, s_bulk=rates.s_bulk,
                        s3=rates.s3, s_high=rates.s_h, m30=m30, D0=D0, D2=D2, adv_u=adv, u_bound=u_bound,
                        dev_bound=dev_bound, gn_bt=gn_bt, gn_dd=gn_dd, src_q=src_q, src_k=src_k,
                        three_level=three_level, mass_src=mass_src, g_share=g_share, lambda1=lambda1,
                        lambda2=lambda2, m2g_form=m2g_form)


def hip_lattice(card):
    from paper_2512_16230_amd import _mrtlb as H
    return H.Lattice(card.kind, card.c, card.cs2, card.free)


def max_rel(a, b):
    """max |a - b| / max |b| (vector fields: magnitude over the components)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim > 2 and a.shape[0] in (2, 3) and a.shape == b.shape and a.ndim in (3, 4):
        return float(np.sqrt(((a - b) ** 2).sum(0)).max() / np.sqrt((b ** 2).sum(0)).max())
    return float(np.abs(a - b).max() / np.abs(b).max())


def max_rel_dev(a, b, ref):
    """max |a - b| / max |b - ref| for fields close to a constant ref."""
    return float(np.abs(a - b).max() / np.abs(b - ref).max())


def check_errs(storage, r, r_o, v, u_o, tr, tu):
    """Assert max_rel of rho (or phi) and u against their tolerances, after
    printing both errors with the test's id (the measured floors behind the
    FP32 tolerances come from these lines)."""
    er, eu = max_rel(r, r_o), max_rel(v, u_o)
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    print("errs %s %s rho %.3e u %.3e (tol %.1e %.1e)" % (test, storage, er, eu, tr, tu), flush=True)
    assert er < tr and eu < tu, (storage, er, eu)
