"""Mixed precision against the FP64 oracle: the rD2Q25 Taylor-Green
benchmark physics on a 256 x 256 box (dx/dy = 1.5, Ma = 0.1, tau = 0.6),
1000 steps, for every storage format.  The oracle fields come from
tests/golden/tgv256_refs.npz (written by make_tgv256_references.py, which
calls only oracle/).

  * error vs the oracle (with the N(0, 1e-3^2) velocity perturbation):
    max |a - b| / max |b| for rho and u, and for the pressure part
    max |a - b| / max |b - 1|;
  * L2 error vs the analytic decaying vortex (no perturbation), as a ratio to
    the FP64 oracle's own L2 error.

The stated bar for a 16-bit format is <= 1e-3 relative error on rho and u and
an L2 ratio <= 1.1.  The int16 fixed-point deviations (ranges sized from the
flow bounds) meet it; FP16 and BF16 deviations, whose 11- and 8-bit
significands are relative to each value, do not: they are bounded here as
measured, with a margin, so that a regression still shows.
"""

import os

import numpy as np
import pytest

from paper_2512_16230_amd import _mrtlb as H
from paper_2512_16230_amd import workloads as W

from helpers import hip_lattice, hip_model, max_rel, max_rel_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.abspath(__file__))
STORAGES = ["fp64", "fp32", "fp32_dev", "fp32_dev_f64", "fp16_dev", "bf16_dev", "i16_dev"]


@pytest.fixture(scope="module")
def refs():
    return np.load(os.path.join(ROOT, "golden", "tgv256_refs.npz"))


@pytest.fixture(scope="module")
def results(refs):
    ctx = H.Context(0)
    shape = tuple(int(v) for v in refs["shape"])
    steps = int(refs["steps"])
    out = {}
    for sigma, tag in ((1e-3, "noise"), (0.0, "clean")):
        wl = W.tgv_large(0, shape=shape, steps=steps, sigma=sigma)
        for storage in STORAGES:
            print("case: tgv-rD2Q25-256x256 %s %s %d steps" % (storage, tag, steps), flush=True)
            bounds = {}
            if storage == "i16_dev":
                ub, db = W.flow_bounds(wl.eq, wl.rho_or_phi, wl.u)
                bounds = {"u_bound": ub, "dev_bound": db}
            s = H.Solve(ctx, hip_lattice(wl.card), hip_model(wl.eq, wl.rates, **bounds), shape, storage)
            s.init_fields(wl.rho_or_phi, wl.u)
            s.step(steps)
            out[(storage, tag)] = s.read_moments()
            s.close()
    ctx.close()
    return out


def _analytic(shape, steps):
    card = W.Q25_RECT
    nu = card.cs2 * (0.6 - 0.5)
    _, ua = W.taylor_green_2d(card, shape, 0.1 * np.sqrt(card.cs2), t=steps, nu=nu)
    return ua


def test_error_against_oracle(refs, results):
    rows = {}
    for storage in STORAGES:
        rho, u = results[(storage, "noise")]
        rows[storage] = (max_rel(rho, refs["rho_noise"]), max_rel_dev(rho, refs["rho_noise"], 1.0),
                         max_rel(u, refs["u_noise"]))
    for k, v in rows.items():
        print("%-9s rho %.2e  rho-1 %.2e  u %.2e" % ((k,) + v), flush=True)
    assert max(rows["fp64"]) < 1e-10
    # the pressure part rho - 1 (max |rho - 1| ~ 0.01): plain FP32 and the
    # 16-bit storages round a density of ~1, so this relative error is ~100x
    # that of rho; FP32 deviations store rho - 1 itself
    assert rows["fp32_dev"][1] < 1e-4
    assert rows["fp32"][1] < 5e-3 and rows["i16_dev"][1] < 5e-3
    # FP32 floor (see test_gpu_parity): measured 9.4e-6 / 4.7e-5 and 3.1e-7 / 3.3e-5
    assert rows["fp32"][0] < 3e-5 and rows["fp32"][2] < 1.5e-4
    assert rows["fp32_dev"][0] < 1e-6 and rows["fp32_dev"][2] < 1e-4
    # FP32 deviations with FP64 arithmetic: only the stored values round
    # (measured rho 3.2e-9, rho - 1 7.6e-7, u 4.0e-8)
    assert rows["fp32_dev_f64"][0] < 1e-8 and rows["fp32_dev_f64"][1] < 2.3e-6 and rows["fp32_dev_f64"][2] < 1.2e-7
    # the stated bar, met by the int16 fixed-point deviations
    assert rows["i16_dev"][0] < 1e-3 and rows["i16_dev"][2] < 1e-3
    # FP16 / BF16 deviations miss it (measured u 2.3e-3 and 3.8e-2)
    assert rows["fp16_dev"][0] < 1e-3 and rows["fp16_dev"][2] < 6e-3
    assert rows["bf16_dev"][0] < 2e-3 and rows["bf16_dev"][2] < 8e-2


def test_l2_against_analytic_within_fp64(refs, results):
    shape = tuple(int(v) for v in refs["shape"])
    ua = _analytic(shape, int(refs["steps"]))
    l2 = lambda u: float(np.sqrt(((u - ua) ** 2).sum() / (ua ** 2).sum()))  # noqa: E731
    base = l2(refs["u_clean"])
    ratios = {st: l2(results[(st, "clean")][1]) / base for st in STORAGES}
    print("oracle L2 vs analytic %.3e; ratios %s" % (base, {k: round(v, 4) for k, v in ratios.items()}), flush=True)
    assert abs(ratios["fp64"] - 1) < 1e-6
    for st in ("fp32", "fp32_dev", "fp32_dev_f64", "i16_dev"):
        assert ratios[st] < 1.1, st
    assert ratios["fp16_dev"] < 4 and ratios["bf16_dev"] < 130


@pytest.mark.parametrize("card,shape", [(W.Q25_RECT, (8, 512)), (W.Q25_RECT, (24, 40)), (W.Q53_RECT, (6, 8, 12))],
                         ids=["rD2Q25-4-nodes-per-thread", "rD2Q25-1-node-per-thread", "rD3Q53"])
def test_int16_saturation_is_reported(card, shape):
    """A uniform body force accelerates a resting fluid past the u_bound its
    int16 ranges were sized for: the next synchronous read returns ENUMERIC
    (the kernels clamp and flag, they never fault), and a solve whose bounds
    cover the run reports nothing."""
    ctx = H.Context(0)
    d = card.d
    rho = np.ones(shape)
    u = np.zeros((d,) + shape)
    F = np.zeros((d,) + shape)
    F[0] = 2e-4
    steps = 400                                  # u grows to F t / rho = 0.08
    rates = W.Rates(1.2, 1.2, 1.25, 1.2, 1.2, 1.2)
    m30 = True
    tight = hip_model("NSE_INC", rates, m30=m30, u_bound=0.005, dev_bound=1e-3)
    print("case: int16 saturation %s %s" % (card.kind, shape), flush=True)
    s = H.Solve(ctx, hip_lattice(card), tight, shape, "i16_dev", has_force=True)
    s.init_fields(rho, u, F)
    s.read_moments()                             # within range at rest
    s.step(steps)
    with pytest.raises(H.MrtlbError) as e:
        s.read_moments()
    assert e.value.status == H.MRTLB_ENUMERIC and "saturated" in str(e.value)
    with pytest.raises(H.MrtlbError) as e:
        s.conserved()
    assert e.value.status == H.MRTLB_ENUMERIC
    s.init_fields(rho, u, F)                     # a new state clears the flag
    s.read_moments()
    s.close()
    ub, db = W.flow_bounds("NSE_INC", rho, u, F, steps, cs2=card.cs2)
    ok = H.Solve(ctx, hip_lattice(card), hip_model("NSE_INC", rates, m30=m30, u_bound=ub, dev_bound=db), shape,
                 "i16_dev", has_force=True)
    ok.init_fields(rho, u, F)
    ok.step(steps)
    r, v = ok.read_moments()
    assert abs(v[0].mean() - 2e-4 * steps) < 1e-3 * 2e-4 * steps
    ok.close()
    ctx.close()
