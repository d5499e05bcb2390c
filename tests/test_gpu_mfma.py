"""The matrix-core (MFMA) Hermite transform, mrtlb_solve_set_transform:
3D lattices with int16 deviation storage, NSE models.

  * against the FP64 oracle on ragged grids (row pitch 64 and 128, idle
    padding slots), at the int16 storage's tolerance, and against the VALU
    transform of the same solve;
  * in the launch configuration of the benchmark (rD3Q53 256^3 compressible
    Taylor-Green): sampled nodes against the oracle on their dependency cones;
  * batched launches of MFMA solves equal their solo runs bit for bit, and a
    solve may switch transforms between steps;
  * the cases outside the MFMA kernel are refused (EINVAL).
"""

import numpy as np
import pytest

from oracle import model as OM
from paper_2512_16230_amd import _mrtlb as H
from paper_2512_16230_amd import workloads as W

from helpers import hip_lattice, hip_model, max_rel, oracle_for

pytestmark = pytest.mark.gpu

CARDS = [W.Q53_RECT, W.Q45_RECT, W.Q33_CUBIC, W.Q27_RECT]


@pytest.fixture(scope="module")
def ctx():
    c = H.Context(0)
    yield c
    c.close()


def _fields(card, shape, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    rho = 1 + amp * rng.normal(size=shape)
    u = amp * rng.normal(size=(3,) + tuple(shape))
    return rho, u


def _run(ctx, card, eq, rates, shape, rho, u, steps, transform, m30):
    ub, db = W.flow_bounds(eq, rho, u, None, steps, cs2=card.cs2)
    s = H.Solve(ctx, hip_lattice(card), hip_model(eq, rates, m30=m30, u_bound=ub, dev_bound=db), shape, "i16_dev")
    s.set_transform(transform)
    s.init_fields(rho, u)
    s.step(steps)
    r, v = s.read_moments()
    s.close()
    return r, v


@pytest.mark.parametrize("card", CARDS, ids=lambda c: c.kind)
@pytest.mark.parametrize("eq", ["NSE_INC", "NSE_COMP"])
@pytest.mark.parametrize("shape", [(6, 10, 64), (5, 7, 100)], ids=["pitch64", "pitch128-ragged"])
def test_mfma_matches_oracle(ctx, card, eq, shape):
    rates = W.Rates(1.1, 1.3, 1.6, 1.05, 1.4, 0.9)
    rho, u = _fields(card, shape, 41)
    steps = 12
    m30 = card.kind != "D3Q27"
    lat, mdl = oracle_for(card, eq, rates, m30=m30)
    st = OM.run(lat, mdl, OM.init_state(lat, mdl, rho, u), steps)
    r_o, u_o = OM.moments(lat, mdl, st)
    print("case: mfma %s %s %s" % (card.kind, eq, shape), flush=True)
    rv, vv = _run(ctx, card, eq, rates, shape, rho, u, steps, "valu", m30)
    rm, vm = _run(ctx, card, eq, rates, shape, rho, u, steps, "mfma", m30)
    ev = (max_rel(rv, r_o), max_rel(vv, u_o))
    em = (max_rel(rm, r_o), max_rel(vm, u_o))
    print("errs %s %s %s: valu rho %.3e u %.3e, mfma rho %.3e u %.3e, mfma-valu rho %.3e u %.3e"
          % (card.kind, eq, shape, ev[0], ev[1], em[0], em[1], max_rel(rm, rv), max_rel(vm, vv)), flush=True)
    assert em[0] < 1e-4 and em[1] < 1e-2
    # the two transforms differ by rounding: within the int16 error of either
    assert em[1] < 3 * ev[1] + 1e-4


def test_full_size_sampled_mfma(ctx):
    """rD3Q53 256^3 compressible Taylor-Green, int16, MFMA transform, in the
    benchmark's launch configuration: sampled nodes after 3 steps against the
    oracle on crops that cover their dependency cones."""
    from test_gpu_parity import _crop3

    wl = W.tgv3d(shape=(256, 256, 256), steps=3)
    steps = 3
    ub, db = W.flow_bounds(wl.eq, wl.rho_or_phi, wl.u, None, steps, cs2=wl.card.cs2)
    print("case: tgv3d-rD3Q53-256^3 i16_dev mfma sampled", flush=True)
    s = H.Solve(ctx, hip_lattice(wl.card), hip_model(wl.eq, wl.rates, u_bound=ub, dev_bound=db), wl.shape,
                "i16_dev")
    s.set_transform("mfma")
    s.init_fields(wl.rho_or_phi, wl.u)
    s.step(steps)
    r, v = s.read_moments()
    s.close()
    rng = np.random.default_rng(1)
    R = 2 * steps + 1
    lat, mdl = oracle_for(wl.card, wl.eq, wl.rates)
    pts = [(0, 0, 0), (255, 255, 255), (128, 3, 250)] + [tuple(rng.integers(0, 256, 3)) for _ in range(3)]
    U0 = wl.meta["U0"]
    er = eu = 0.0
    for iz, iy, ix in pts:
        st = OM.run(lat, mdl, OM.init_state(lat, mdl, _crop3(wl.rho_or_phi, iz, iy, ix, R),
                                            _crop3(wl.u, iz, iy, ix, R)), steps)
        ro, uo = OM.moments(lat, mdl, st)
        er = max(er, abs(r[iz, iy, ix] - ro[R, R, R]) / abs(ro[R, R, R]))
        eu = max(eu, np.abs(v[:, iz, iy, ix] - uo[:, R, R, R]).max() / U0)
    print("sampled errors: rho %.3e, u %.3e of U0" % (er, eu), flush=True)
    assert er < 1e-5 and eu < 1e-3


def test_mfma_batch_and_switch(ctx):
    card = W.Q53_RECT
    rates = W.Rates(1.1, 1.3, 1.6, 1.05, 1.4, 0.9)
    shapes = [(6, 10, 64), (5, 7, 100), (4, 6, 128)]
    solo, batch = [], []
    for k, shape in enumerate(shapes):
        rho, u = _fields(card, shape, 50 + k)
        ub, db = W.flow_bounds("NSE_COMP", rho, u, None, 20, cs2=card.cs2)
        for lst in (solo, batch):
            s = H.Solve(ctx, hip_lattice(card), hip_model("NSE_COMP", rates, u_bound=ub, dev_bound=db), shape,
                        "i16_dev")
            s.set_transform("mfma")
            s.init_fields(rho, u)
            lst.append(s)
    counts = [9, 4, 7]
    for s, n in zip(solo, counts):
        s.step(n)
    H.batch_step(batch, counts)
    for a, b in zip(solo, batch):
        assert np.array_equal(a.read_populations(), b.read_populations())
    # switching transforms keeps the stored format: a few VALU steps then MFMA again
    a = solo[0]
    a.set_transform("valu")
    a.step(3)
    a.set_transform("mfma")
    a.step(3)
    a.read_moments()
    for s in solo + batch:
        s.close()


def test_mfma_refuses_other_cases(ctx):
    rates = W.Rates()
    cases = [
        (W.Q25_RECT, (8, 64), "i16_dev", "NSE_INC", False),      # 2D lattice
        (W.Q53_RECT, (6, 10, 64), "fp32", "NSE_INC", False),     # storage
        (W.Q53_RECT, (6, 10, 64), "i16_dev", "NSE_INC", True),   # force field
        (W.Q53_RECT, (6, 10, 90), "i16_dev", "NSE_INC", False),  # row pitch 96
    ]
    for card, shape, storage, eq, forced in cases:
        s = H.Solve(ctx, hip_lattice(card), hip_model(eq, rates), shape, storage, has_force=forced)
        with pytest.raises(H.MrtlbError) as e:
            s.set_transform("mfma")
        assert e.value.status == H.MRTLB_EINVAL
        s.close()
