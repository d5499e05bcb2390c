"""Pins of the standard-lattice (k = 1) path of the oracle: D2Q9 and D3Q27
with the non-diagonal S2 block of eqs. (4-27), (4-27-1).

  * the weights reduce to the textbook D2Q9 / D3Q27 weights on the square
    lattice with cs^2 = 1/3, and on the rectangular cards they meet the
    moment conditions the single layer can meet;
  * on the isotropic square lattice (c_a^2 = 3 cs^2) the S2 block is the
    plain trace/deviator split: bulk rate on the trace, shear rate on the
    deviator;
  * dynamics on the rectangular D2Q9 (dx/dy = 1.5, cs^2 = 1/2, so
    c_x^2 - cs^2 = 3.5 cs^2 and c_y^2 - cs^2 = cs^2, far from isotropic):
    shear-wave decay nu k^2, sound damping (k^2/2)(nu + nu_b) along both
    axes (on D3Q27, 1 : 1.25 : 1.5, along x and z with 4 nu / 3 + nu_b), Taylor-Green decay nu (kx^2 + ky^2), with the viscosities the
    multispeed lattices get from the same s_shear and s_bulk.  A planted
    isotropic block (the multispeed relaxation put on D2Q9) misses the
    sound damping by tens of percent, so the test sees the block;
  * the vectorised reduced form equals the explicit b x b collision.
"""

import numpy as np
import pytest
from scipy.optimize import curve_fit

from oracle import lattice as L
from oracle import model as M
from oracle import naive as N
import test_oracle_collision as C
from paper_2512_16230_amd import workloads as W


def lat_of(card):
    return L.make_lattice(card.kind, card.c, card.cs2, card.free)


@pytest.mark.parametrize("card", [W.Q9_RECT, W.Q27_RECT], ids=lambda c: c.kind)
@pytest.mark.parametrize("eq", [M.NSE_INC, M.NSE_COMP])
def test_equilibrium_moments(card, eq):
    """k = 1, M30 = 0 (standard-lattice case of Sec. IV-B): M0..M2 exact,
    mixed third moments p Delta.u; the pure third moments are what a single
    layer gives, c_a^2 rho u_a."""
    lat = lat_of(card)
    rng = np.random.default_rng(8)
    n, d, cs2, rho0 = 6, lat.d, lat.cs2, 1.3
    R0, u = C._random_state(lat, n, rng)
    mdl = M.Model(eq=eq, rho0=rho0, m30=False)
    rho = np.full(n, rho0) if eq == M.NSE_INC else R0
    feq = M.populations_from_hermite(lat, M.equilibrium_hermite(lat, mdl, R0, u, rho))
    m0, m1, m2, m3 = C._tensor_moments(lat, feq)
    p = cs2 * R0
    assert np.allclose(m0, R0, atol=1e-13)
    assert np.allclose(m1, rho * u, atol=1e-13)
    assert np.allclose(m2, np.einsum("n,an,bn->abn", rho, u, u) + p * np.eye(d)[:, :, None], atol=1e-13)
    visc = (p if eq == M.NSE_COMP else rho * cs2) * C._delta_u(d, u)
    for a in range(d):
        for b in range(d):
            for c in range(d):
                if a == b == c:
                    assert np.allclose(m3[a, a, a], card.c[a] ** 2 * rho * u[a], atol=1e-13)
                else:
                    assert np.allclose(m3[a, b, c], visc[a, b, c], atol=1e-13)


def test_textbook_weights_on_the_square_lattice():
    q9 = L.make_lattice("D2Q9", (1.0, 1.0), 1 / 3)
    assert np.allclose(q9.w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-15)
    q27 = L.make_lattice("D3Q27", (1.0, 1.0, 1.0), 1 / 3)
    layer = np.abs(q27.e).sum(axis=1)
    ref = np.array([8 / 27, 2 / 27, 1 / 54, 1 / 216])[layer]
    assert np.allclose(q27.w, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("card", [W.Q9_RECT, W.Q27_RECT], ids=lambda c: c.kind)
def test_rectangular_weights_meet_the_moment_conditions(card):
    lat = lat_of(card)
    E, w, cs2, d = lat.E, lat.w, lat.cs2, lat.d
    assert (w > 0).all()
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("j,ja,jb->ab", w, E, E), cs2 * np.eye(d), atol=1e-15)
    assert np.abs(np.einsum("j,ja->a", w, E)).max() < 1e-15
    assert np.abs(np.einsum("j,ja,jb,jc->abc", w, E, E, E)).max() < 1e-15
    for a in range(d):
        for b in range(d):
            m4 = (w * E[:, a] ** 2 * E[:, b] ** 2).sum()
            assert abs(m4 - (cs2 * card.c[a] ** 2 if a == b else cs2 ** 2)) < 1e-14
    # rows of order <= 3 are W-orthogonal and there is no pure third-order row
    H = lat.H()
    G = (H * w) @ H.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-13
    assert not [r for r in lat.rows if r.order == 3 and len(set(r.name)) == 1]
    assert len(lat.rows) == (8 if d == 2 else 17)


@pytest.mark.parametrize("kind,c", [("D2Q9", (1.0, 1.0)), ("D3Q27", (1.0, 1.0, 1.0))])
def test_s2_block_is_trace_deviator_on_the_isotropic_lattice(kind, c):
    lat = L.make_lattice(kind, c, 1 / 3)
    mdl = M.Model(eq=M.NSE_COMP, s_shear=1.4, s_bulk=0.9)
    d = lat.d
    P = np.full((d, d), 1.0 / d)
    ref = mdl.s_bulk * P + mdl.s_shear * (np.eye(d) - P)
    assert np.allclose(M.s2_normal_block(lat, mdl), ref, rtol=0, atol=1e-14)


def _sound_rate(card, axis, n=48, steps=240, eps=1e-4):
    """Fitted damping rate of a standing sound wave along ``axis``."""
    lat = lat_of(card)
    d = lat.d
    mdl = M.Model(eq=M.NSE_COMP, s_shear=1.25, s_bulk=1.2, s3=1.1, s_h=1.1)
    shape = [1] * d
    shape[d - 1 - axis] = n
    shape = tuple(shape)
    k = 2 * np.pi / (n * card.c[axis])
    x = W.axis_coords(card, shape, axis) * np.ones(shape)
    rho = 1 + eps * np.cos(k * x)
    st = M.init_state(lat, mdl, rho, np.zeros((d,) + shape))
    amp = []
    for _ in range(steps):
        r, _ = M.moments(lat, mdl, st)
        amp.append(((r - 1) * np.cos(k * x)).sum() / (0.5 * n * eps))
        st = M.step(lat, mdl, st)
    t = np.arange(steps, dtype=np.float64)
    fit = lambda t, A, g, om, ph: A * np.exp(-g * t) * np.cos(om * t + ph)  # noqa: E731
    p, _ = curve_fit(fit, t, np.array(amp), p0=(1.0, 1e-3, np.sqrt(lat.cs2) * k, 0.0))
    nu = lat.cs2 * (1 / mdl.s_shear - 0.5)
    nu_b = (2 / d) * lat.cs2 * (1 / mdl.s_bulk - 0.5)
    # longitudinal viscosity 2 nu (1 - 1/d) + nu_b
    return p[1] / (0.5 * k * k * (2 * nu * (1 - 1 / d) + nu_b)), p[2] / (np.sqrt(lat.cs2) * k)


@pytest.mark.parametrize("card,axis", [(W.Q9_RECT, 0), (W.Q9_RECT, 1), (W.Q27_RECT, 0), (W.Q27_RECT, 2)],
                         ids=["D2Q9-x", "D2Q9-y", "D3Q27-x", "D3Q27-z"])
def test_sound_damping_on_rectangular_lattices(card, axis):
    ratio, speed = _sound_rate(card, axis)
    assert abs(ratio - 1) < 0.005
    assert abs(speed - 1) < 0.005


@pytest.mark.parametrize("axis", [0, 1])
def test_planted_isotropic_block_misses_the_sound_damping(axis, monkeypatch):
    def isotropic(lat, mdl):
        P = np.full((lat.d, lat.d), 1.0 / lat.d)
        return mdl.s_bulk * P + mdl.s_shear * (np.eye(lat.d) - P)

    monkeypatch.setattr(M, "s2_normal_block", isotropic)
    ratio, _ = _sound_rate(W.Q9_RECT, axis)
    assert abs(ratio - 1) > 0.2


def test_shear_wave_decay_on_rectangular_d2q9():
    card = W.Q9_RECT
    lat = lat_of(card)
    mdl = M.Model(eq=M.NSE_INC, s_shear=1.25, s_bulk=1.2, s3=1.1, s_h=1.1)
    n, steps, U = 48, 300, 1e-3
    shape = (n, 1)
    k = 2 * np.pi / (n * card.c[1])
    y = W.axis_coords(card, shape, 1) * np.ones(shape)
    u = np.stack([U * np.sin(k * y), np.zeros(shape)])
    st = M.init_state(lat, mdl, np.ones(shape), u)
    amp = []
    for _ in range(steps):
        _, uu = M.moments(lat, mdl, st)
        amp.append((uu[0] * np.sin(k * y)).sum())
        st = M.step(lat, mdl, st)
    rate = -np.polyfit(np.arange(20, steps), np.log(amp[20:]), 1)[0]
    nu = lat.cs2 * (1 / mdl.s_shear - 0.5)
    assert abs(rate / (nu * k * k) - 1) < 0.01


def test_taylor_green_decay_on_rectangular_d2q9():
    card = W.Q9_RECT
    lat = lat_of(card)
    mdl = M.Model(eq=M.NSE_INC, s_shear=1.25, s_bulk=1.2, s3=1.1, s_h=1.1)
    shape, steps = (48, 32), 300          # equal box lengths: 48 * 1.0 = 32 * 1.5
    p, u = W.taylor_green_2d(card, shape, 1e-3)
    st = M.init_state(lat, mdl, 1.0 + p / lat.cs2, u)
    E = []
    for _ in range(steps):
        _, uu = M.moments(lat, mdl, st)
        E.append((uu ** 2).sum())
        st = M.step(lat, mdl, st)
    rate = -np.polyfit(np.arange(20, steps), np.log(E[20:]), 1)[0] / 2
    kx = 2 * np.pi / (shape[1] * card.c[0])
    ky = 2 * np.pi / (shape[0] * card.c[1])
    nu = lat.cs2 * (1 / mdl.s_shear - 0.5)
    assert abs(rate / (nu * (kx * kx + ky * ky)) - 1) < 0.01


@pytest.mark.parametrize("card,eq,shape", [
    (W.Q9_RECT, M.NSE_INC, (4, 3)),
    (W.Q9_RECT, M.NSE_COMP, (3, 5)),
    (W.Q27_RECT, M.NSE_COMP, (2, 3, 2)),
], ids=lambda v: getattr(v, "kind", str(v)))
def test_vectorised_step_equals_brute_force(card, eq, shape):
    lat = lat_of(card)
    rng = np.random.default_rng(21)
    d = lat.d
    mdl = M.Model(eq=eq, s0=1.1, s1=1.15, s_shear=1.6, s_bulk=1.05, s3=1.4, s_h=0.9, m30=False)
    rho = 1 + 0.05 * rng.normal(size=shape)
    u = 0.05 * rng.normal(size=(d,) + shape)
    F = 1e-3 * rng.normal(size=(d,) + shape)
    st = M.init_state(lat, mdl, rho, u, F)
    st.f = st.f + 1e-3 * rng.normal(size=st.f.shape) * lat.w.reshape((-1,) + (1,) * len(shape))
    nv = N.NaiveStepper(lat, mdl)
    a = st
    b = M.State(st.f.copy())
    for _ in range(3):
        a = M.step(lat, mdl, a, F)
        b = nv.step(b, F)
    assert np.abs(a.f - b.f).max() < 1e-13
