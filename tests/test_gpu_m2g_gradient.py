"""GPU parity of the mass-source field and of the gradient form of M2G_bar
(eqs. M2G, M2G-1): the HIP library through its C ABI against the FP64
oracle run on the same sequence of forces and sources, and the physics
pins of the oracle (a hydrostatic stream, a uniformly translating
incompressible fluid with a source) on the GPU.

Tolerances as in test_gpu_parity: FP64 differs from the oracle only in the
rounding order; FP32 bounds are at most 3x the measured error of each case
(printed by check_errs).
"""

import numpy as np
import pytest

from oracle import model as OM
from paper_2512_16230_amd import _mrtlb as H
from paper_2512_16230_amd import workloads as W

from helpers import check_errs, hip_lattice, hip_model, oracle_for
import test_oracle_m2g_gradient as TG

pytestmark = pytest.mark.gpu

RATES = W.Rates(1.6, 1.3, 1.25, 1.1, 1.15, 1.2)


@pytest.fixture(scope="module")
def ctx():
    c = H.Context(0)
    yield c
    c.close()


def _fields(card, shape, seed):
    rng = np.random.default_rng(seed)
    d = card.d
    rho = 1 + 0.02 * rng.normal(size=shape)
    u = 0.03 * rng.normal(size=(d,) + tuple(shape))
    F = W.sinusoidal_force(card, shape, 1e-3, seed=seed + 1)
    S = [1e-4 * (1 + rng.random(shape)) for _ in range(12)]
    return rho, u, F, S


def _run_pair(ctx, card, shape, eq, kw, storage, steps, forced, seed=21):
    """(oracle rho, u, totals) and (GPU rho, u, totals) after ``steps`` steps
    with the mass-source field changing every step (forced runs) or plain."""
    rho, u, F, S = _fields(card, shape, seed)
    Fk = (lambda k: F * (1 + 0.2 * k)) if forced else (lambda k: None)
    lat, mdl = oracle_for(card, eq, RATES, **kw)
    if forced:
        mdl.mass_src = S[0]
    st = OM.init_state(lat, mdl, rho, u, Fk(0))
    for k in range(steps):
        if forced:
            mdl.mass_src = S[k]
        st = OM.step(lat, mdl, st, Fk(k))
    if forced:
        mdl.mass_src = S[steps]
    r_o, u_o = OM.moments(lat, mdl, st, Fk(steps))
    tot_o = OM.conserved(lat, mdl, st, Fk(steps))
    s = H.Solve(ctx, hip_lattice(card), hip_model(eq, RATES, **kw), shape, storage, has_force=forced)
    if forced:
        s.set_mass_source_field(S[0])
    s.init_fields(rho, u, Fk(0))
    for k in range(steps):
        if forced:
            s.set_force_field(Fk(k))
            s.set_mass_source_field(S[k])
        s.step(1)
    if forced:
        s.set_force_field(Fk(steps))
        s.set_mass_source_field(S[steps])
    r, v = s.read_moments()
    tot = s.conserved()
    s.close()
    return (r_o, u_o, tot_o), (r, v, tot)


CASES = [(W.Q25_RECT, (12, 70), "NSE_INC"), (W.Q25_RECT, (12, 70), "NSE_COMP"),
         (W.Q53_RECT, (6, 10, 40), "NSE_INC"), (W.Q53_RECT, (6, 10, 40), "NSE_COMP"),
         (W.Q9_RECT, (37, 66), "NSE_INC")]
# FP32 and FP32-storage/FP64-arithmetic bounds per lattice: 3x the largest
# (rho, u) error measured over its cases
TOL = {"rD2Q25": {"fp32": (6.5e-7, 3.8e-5), "fp32_dev_f64": (1e-9, 7.5e-8)},
       "rD3Q53": {"fp32": (4.6e-7, 6.6e-5), "fp32_dev_f64": (5e-10, 8.1e-8)},
       "D2Q9": {"fp32": (1.2e-6, 1.8e-5), "fp32_dev_f64": (7.9e-9, 1.1e-7)}}


@pytest.mark.parametrize("card,shape,eq", CASES, ids=lambda v: getattr(v, "kind", v if isinstance(v, str) else "x"))
@pytest.mark.parametrize("forced", [False, True], ids=["plain", "force-and-source-field"])
def test_gradient_form_matches_oracle(ctx, card, shape, eq, forced):
    kw = dict(m2g_form=1, m30=card.kind not in ("D2Q9", "D3Q27"))
    t = TOL[card.kind]
    for storage, tr, tu in (("fp64", 3e-14, 5e-13), ("fp32",) + t["fp32"], ("fp32_dev_f64",) + t["fp32_dev_f64"]):
        print("case: gradient form %s %s %s forced=%s %s" % (card.kind, shape, eq, forced, storage), flush=True)
        (r_o, u_o, (m_o, p_o)), (r, v, (m, p)) = _run_pair(ctx, card, shape, eq, kw, storage, 10, forced)
        check_errs(storage, r, r_o, v, u_o, tr, tu)
        tol = 1e-12 if storage == "fp64" else 1e-6
        assert abs(m - m_o) < tol * abs(m_o) and np.abs(p - p_o).max() < tol * abs(m_o)


@pytest.mark.parametrize("card,shape", [(W.Q25_RECT, (12, 70)), (W.Q53_RECT, (6, 10, 40))], ids=["rD2Q25", "rD3Q53"])
@pytest.mark.parametrize("scheme", ["closed", "three-level", "split"])
def test_mass_source_field_matches_oracle(ctx, card, shape, scheme):
    """The closed form with a source field S(x, t): the F route, the
    three-level scheme (the source's difference term) and a share in G."""
    kw = {"closed": dict(), "three-level": dict(three_level=True),
          "split": dict(g_share=0.4, lambda1=0.7, lambda2=1.2)}[scheme]
    # FP32: 3x the largest error measured over the schemes per lattice
    t32 = {"rD2Q25": (7.5e-7, 3.1e-5), "rD3Q53": (5.2e-7, 3.7e-5)}[card.kind]
    for storage, tr, tu in (("fp64", 3e-14, 5e-13), ("fp32",) + t32):
        print("case: source field %s %s %s" % (scheme, card.kind, storage), flush=True)
        (r_o, u_o, (m_o, _)), (r, v, (m, _)) = _run_pair(ctx, card, shape, "NSE_COMP", kw, storage, 10, True)
        check_errs(storage, r, r_o, v, u_o, tr, tu)
        assert abs(m - m_o) < (1e-12 if storage == "fp64" else 1e-6) * abs(m_o)


@pytest.mark.parametrize("card", [W.Q25_RECT, W.Q9_RECT], ids=lambda c: c.kind)
def test_hydrostatic_stream_on_the_gpu(ctx, card):
    """The oracle's steady stratified stream, on the GPU in FP64: the
    gradient form keeps U (measured in the oracle 2.5e-5 rD2Q25, 3.7e-6
    D2Q9); the closed form drifts 20x more."""
    ny, nx = 32, 4
    y = np.arange(ny)[:, None] * card.c[1]
    k = 2 * np.pi / (ny * card.c[1])
    U = 0.1 * np.sqrt(card.cs2)
    rho = (1 + 0.01 * np.cos(k * y)) * np.ones((1, nx))
    fy = card.cs2 * (np.roll(rho, -1, axis=0) - np.roll(rho, 1, axis=0)) / (2 * card.c[1])
    F = np.stack([np.zeros_like(rho), fy])
    u = np.stack([np.full_like(rho, U), np.zeros_like(rho)])
    drift = []
    for form in (0, 1):
        s = H.Solve(ctx, hip_lattice(card), hip_model("NSE_INC", RATES, m2g_form=form,
                                                      m30=card.kind not in ("D2Q9", "D3Q27")),
                    (ny, nx), "fp64", has_force=True)
        s.init_fields(rho, u, F)
        s.step(300)
        _, v = s.read_moments()
        drift.append(float(np.abs(v[0] - U).max()))
        s.close()
    want = TG.stratified_stream(card, 1, False)
    print("hydrostatic stream %s: closed %.3e gradient %.3e (oracle %.3e)" % (card.kind, drift[0], drift[1], want),
          flush=True)
    assert abs(drift[1] - want) < 1e-12 and drift[0] > 20 * drift[1]


@pytest.mark.parametrize("card", [W.Q25_RECT, W.Q53_RECT, W.Q9_RECT], ids=lambda c: c.kind)
def test_uniform_incompressible_source_shear_on_the_gpu(ctx, card):
    """The oracle's uniformly translating NSE_INC fluid with a uniform source,
    on the GPU in FP64: the off-diagonal non-equilibrium second moment is 0
    with the gradient form and (1/2 - 1/s_shear) u_x u_y S with the closed form."""
    d = card.d
    shape = (3,) * d
    U = np.array([0.05, -0.03, 0.02])[:d]
    u = np.stack([np.full(shape, U[a]) for a in range(d)])
    got = []
    for form in (0, 1):
        s = H.Solve(ctx, hip_lattice(card), hip_model("NSE_INC", RATES, mass_src=2e-4, m2g_form=form,
                                                      m30=card.kind not in ("D2Q9", "D3Q27")),
                    shape, "fp64", has_force=True)
        s.init_fields(np.ones(shape), u, np.zeros((d,) + shape))
        s.step(60)
        f = s.read_populations().reshape(card_b(card), -1)[:, 0]
        s.close()
        E = np.array(hip_lattice_velocities(card), dtype=np.float64)
        got.append(float(np.einsum("j,j,j->", f, E[:, 0], E[:, 1]) - U[0] * U[1]))
    want = [TG.uniform_inc_source_shear(card, form) for form in (0, 1)]
    print("uniform source shear %s: closed %.3e (oracle %.3e) gradient %.3e" % (card.kind, got[0], want[0], got[1]),
          flush=True)
    # the sum over b populations of size ~0.1 rounds at ~1e-16
    assert abs(got[0] - want[0]) < 1e-15 and abs(got[1]) < 1e-15


def card_b(card):
    from oracle import lattice as OL
    return OL.make_lattice(card.kind, card.c, card.cs2, card.free).b


def hip_lattice_velocities(card):
    from oracle import lattice as OL
    return OL.make_lattice(card.kind, card.c, card.cs2, card.free).E


def test_batch_equals_single(ctx):
    card, shape = W.Q25_RECT, (12, 70)
    rho, u, F, S = _fields(card, shape, 5)
    outs = []
    for batched in (False, True):
        s = H.Solve(ctx, hip_lattice(card), hip_model("NSE_COMP", RATES, m2g_form=1), shape, "fp64", has_force=True)
        s.set_mass_source_field(S[0])
        s.init_fields(rho, u, F)
        if batched:
            H.batch_step([s], [7])
        else:
            s.step(7)
        outs.append(s.read_populations())
        s.close()
    assert np.array_equal(outs[0], outs[1])


def test_errors(ctx):
    card, shape = W.Q25_RECT, (16, 16)

    def refused(eq, storage, lat=hip_lattice(card), force=False, **kw):
        with pytest.raises(H.MrtlbError) as e:
            H.Solve(ctx, lat, hip_model(eq, RATES, **kw), shape, storage, has_force=force)
        assert e.value.status == H.MRTLB_EINVAL

    refused("NSE_INC", "fp16_dev", m2g_form=1)
    refused("NSE_COMP", "fp32", lat=hip_lattice(W.Q9_RECT), m2g_form=1)
    refused("NCDE", "fp32", D0=0.1, m2g_form=1)
    refused("NSE_INC", "fp32", m2g_form=2)
    s = H.Solve(ctx, hip_lattice(card), hip_model("NSE_INC", RATES), shape, "fp32")
    with pytest.raises(H.MrtlbError) as e:
        s.set_mass_source_field(np.zeros(shape))
    assert e.value.status == H.MRTLB_EINVAL
    s.close()
    s = H.Solve(ctx, hip_lattice(card), hip_model("NSE_COMP", RATES), shape, "fp32", has_force=True)
    bad = np.zeros(shape)
    bad[2, 2] = np.nan
    with pytest.raises(H.MrtlbError) as e:
        s.set_mass_source_field(bad)
    assert e.value.status == H.MRTLB_ENUMERIC
    s.close()
