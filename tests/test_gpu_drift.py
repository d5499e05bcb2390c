"""Drift correction of the conserved totals (mrtlb_set_drift_correction).

The collision conserves mass (and momentum without a force) exactly; the
rounding of the stored populations does not, and on a smooth flow its
errors add up.  With the correction the FP64 totals are checked every K
steps and the difference is put back on the next step.  Checked here: the
totals stay at their reference, the batched path applies the same
corrections at the same steps (bit for bit), and the accuracy against the
FP64 oracle is unchanged.
"""

import os

import numpy as np
import pytest

from paper_2512_16230_amd import _mrtlb as H
from paper_2512_16230_amd import workloads as W

from helpers import hip_lattice, hip_model, max_rel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx():
    c = H.Context(0)
    yield c
    c.close()


def _solve(ctx, wl, storage, every=0):
    kw = {}
    if storage == "i16_dev":
        ub, db = W.flow_bounds(wl.eq, wl.rho_or_phi, wl.u)
        kw = dict(u_bound=ub, dev_bound=db)
    s = H.Solve(ctx, hip_lattice(wl.card), hip_model(wl.eq, wl.rates, **kw), wl.shape, storage)
    s.init_fields(wl.rho_or_phi, wl.u)
    if every:
        s.set_drift_correction(every)
    return s


@pytest.mark.parametrize("storage", ["fp32", "i16_dev", "fp16_dev"])
def test_totals_held(ctx, storage):
    wl = W.tgv_large(0, shape=(256, 256), steps=3000)
    print("case: tgv-rD2Q25-256x256 %s drift correction every 100, 3000 steps" % storage, flush=True)
    res = {}
    for every in (0, 100):
        s = _solve(ctx, wl, storage, every)
        m0, p0 = s.conserved()
        s.step(3000)
        m1, p1 = s.conserved()
        res[every] = (abs(m1 - m0) / m0, np.abs(p1 - p0).max() / m0)
        s.close()
    print(storage, "without: dm %.2e dp %.2e; with: dm %.2e dp %.2e" % (res[0] + res[100]), flush=True)
    # the last check was at step 3000: the difference it found is still
    # pending, so the state carries at most 100 steps of drift.  The mass
    # drift is systematic and is removed; the 16-bit storages' momentum
    # drift is mostly rounding noise of the last steps, of order 1e-7.
    assert res[100][0] < max(1e-9, 0.2 * res[0][0])
    assert res[100][1] < max(2e-7, 0.2 * res[0][1])


def test_batched_path_applies_the_same_corrections(ctx):
    wl = W.tgv_large(1, shape=(96, 160), steps=250)
    a = _solve(ctx, wl, "i16_dev", every=40)
    b = _solve(ctx, wl, "i16_dev", every=40)
    c = _solve(ctx, wl, "i16_dev", every=0)
    a.step(250)
    # the serving loop's pattern: chunks that do not line up with the checks
    for k in (64, 64, 64, 58):
        H.batch_step([b, c], [k, k])
    fa, fb = a.read_populations(), b.read_populations()
    assert np.array_equal(fa, fb)
    assert not np.array_equal(fa, c.read_populations())
    for s in (a, b, c):
        s.close()


def test_accuracy_kept(ctx):
    refs = np.load(os.path.join(ROOT, "golden", "tgv256_refs.npz"))
    shape = tuple(int(v) for v in refs["shape"])
    steps = int(refs["steps"])
    wl = W.tgv_large(0, shape=shape, steps=steps, sigma=1e-3)
    s = _solve(ctx, wl, "i16_dev", every=100)
    s.step(steps)
    rho, u = s.read_moments()
    s.close()
    e_rho, e_u = max_rel(rho, refs["rho_noise"]), max_rel(u, refs["u_noise"])
    print("i16_dev with drift correction: rho %.2e u %.2e" % (e_rho, e_u), flush=True)
    assert e_rho < 1e-3 and e_u < 1e-3


@pytest.mark.parametrize("s_high", [0.9, 1.5])
def test_one_corrected_step_restores_the_totals(ctx, s_high):
    """After the FP64 check at step K the next step moves the totals back to
    the reference by the whole difference: the rate s_h of the rows above
    third order (which act on the uncorrected populations) must not scale
    it.  FP32 storage drifts systematically; the step after the correction
    keeps at most its own one-step drift."""
    wl = W.tgv_large(0, shape=(256, 256), steps=201)
    r = wl.rates
    wl.rates = W.Rates(r.s0, r.s1, r.s_shear, r.s_bulk, r.s3, s_high)
    K = 200
    print("case: tgv-rD2Q25-256x256 fp32 s_high %.2f, check after %d steps, one corrected step" % (s_high, K),
          flush=True)
    s = _solve(ctx, wl, "fp32", every=K)
    m_ref, p_ref = s.conserved()
    s.step(K)                 # the check at step K finds the drift; the correction is pending
    m_k, p_k = s.conserved()
    s.step(1)
    m_1, p_1 = s.conserved()
    s.close()
    dm, dp = abs(m_k - m_ref), np.abs(p_k - p_ref).max()
    rm, rp = abs(m_1 - m_ref), np.abs(p_1 - p_ref).max()
    print("drift before %.3e / %.3e, after the corrected step %.3e / %.3e" % (dm, dp, rm, rp), flush=True)
    assert dm > 1e-8 * m_ref                  # there is a drift to correct
    assert rm < 0.05 * dm
    assert rp < max(0.05 * dp, 1e-9 * m_ref)
