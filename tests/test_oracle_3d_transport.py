"""Pins of the oracle's convection-diffusion models (NCDE, and its CDE
special case (3)) on the 3D lattices and with a time-dependent velocity.

The NCDE of App. A is d-dimensional: on rD3Q53 (1 : 1.25 : 1.5), rD3Q33
(cubic) and the standard D3Q27 a Gaussian hill with linear D (D2 = 0) and a
constant advection velocity follows the closed form
  phi = A (s0^2 / s^2)^{3/2} exp(-|x - x0 - u t|^2 / (2 s^2)),  s^2 = s0^2 + 2 K t
(periodic images summed, physical positions x = i c), the total of phi is
kept to rounding, and the error falls at second order under refinement.
The CDE (velocity field, S_G = -u . grad phi) follows the same closed form,
also when the velocity changes in time: for a uniform u(t) the hill's centre
moves by the integral of u.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import model as M
from paper_2512_16230_amd import workloads as W


def _lat(card):
    return L.make_lattice(card.kind, card.c, card.cs2, card.free)


def hill_closed_form(card, shape, t, K, shift, s0):
    """Gaussian hill (amplitude 1, width s0, centred) after time t, displaced
    by `shift` (physical), periodic images summed."""
    d = card.d
    Ls = [shape[d - 1 - a] * card.c[a] for a in range(d)]
    s2 = s0 ** 2 + 2 * K * t
    out = (s0 ** 2 / s2) ** (d / 2.0)
    for a in range(d):
        xa = W.axis_coords(card, shape, a)
        c = 0.5 * Ls[a] + shift[a]
        out = out * sum(np.exp(-(xa - c + k * Ls[a]) ** 2 / (2 * s2)) for k in (-2, -1, 0, 1, 2))
    return np.broadcast_to(out, shape)


def _ncde_model(card, wl, D0):
    r = wl.rates
    return M.Model(eq=M.NCDE, s0=r.s0, s1=r.s1, s_shear=r.s_shear, s_bulk=r.s_bulk, s3=r.s3, s_h=r.s_h, D0=D0,
                   D2=0.0, adv_u=wl.adv_u)


def _ncde_3d(card, N, steps, adv=(0.02, -0.015, 0.01), D0f=0.3):
    """Closed-form error and relative mass change of the advected hill, width
    N / 8, K = D0f cs^2."""
    shape = (N, N, N)
    s0, D0 = N / 8.0, D0f * card.cs2
    wl = W.ncde_hill(shape, steps, adv_u=adv, D0=D0, D2=0.0, card=card)
    wl.rho_or_phi = W.gaussian_hill(card, shape, sigma0=s0)
    lat, mdl = _lat(card), _ncde_model(card, wl, D0)
    st = M.init_state(lat, mdl, wl.rho_or_phi)
    m0 = st.f.sum()
    st = M.run(lat, mdl, st, steps)
    phi, _ = M.moments(lat, mdl, st)
    ref = hill_closed_form(card, shape, steps, D0, [adv[a] * steps for a in range(3)], s0)
    return np.abs(phi - ref).max() / ref.max(), (st.f.sum() - m0) / m0


@pytest.mark.parametrize("card", [W.Q53_RECT, W.Q33_CUBIC, W.Q27_RECT], ids=lambda c: c.kind)
def test_ncde_3d_variance_grows_at_2K(card):
    """Resting hill, linear D = K: after the initial layer (10 steps) the
    variance along every axis grows by exactly 2 K per step."""
    shape, s0, D0 = (32, 36, 48), 2.5, 0.2 * card.cs2
    wl = W.ncde_hill(shape, 30, adv_u=(0.0, 0.0, 0.0), D0=D0, D2=0.0, card=card)
    wl.rho_or_phi = W.gaussian_hill(card, shape, sigma0=s0)
    lat, mdl = _lat(card), _ncde_model(card, wl, D0)

    def var(phi):
        out = []
        for a in range(3):
            x = W.axis_coords(card, shape, a) - 0.5 * shape[2 - a] * card.c[a]
            out.append((phi * x ** 2).sum() / phi.sum())
        return np.array(out)

    st = M.run(lat, mdl, M.init_state(lat, mdl, wl.rho_or_phi), 10)
    v0 = var(M.moments(lat, mdl, st)[0])
    st = M.run(lat, mdl, st, 20)
    v1 = var(M.moments(lat, mdl, st)[0])
    assert np.abs((v1 - v0) / (2 * D0 * 20) - 1).max() < 1e-4


@pytest.mark.parametrize("card", [W.Q53_RECT, W.Q27_RECT], ids=lambda c: c.kind)
def test_ncde_3d_gaussian_hill(card):
    err, dm = _ncde_3d(card, 24, 36)
    assert abs(dm) < 1e-13
    assert err < 5e-2


def test_ncde_3d_second_order():
    """rD3Q33 (cubic): N = 16, 9 steps against N = 32, 36 steps (diffusive
    scaling): the closed-form error falls about 4x."""
    e16, _ = _ncde_3d(W.Q33_CUBIC, 16, 9)
    e32, _ = _ncde_3d(W.Q33_CUBIC, 32, 36)
    assert 3.0 < e16 / e32 < 5.5


def _cde_run(card, shape, steps, vel_at, D0, s0):
    """CDE run with the velocity field vel_at(n) (d, *shape) at step n
    (K = D0)."""
    wl = W.cde_hill(shape, steps, u=vel_at(0), D0=D0, card=card)
    wl.rho_or_phi = W.gaussian_hill(card, shape, sigma0=s0)
    lat = _lat(card)
    r = wl.rates
    mdl = M.Model(eq=M.CDE, s0=r.s0, s1=r.s1, s_shear=r.s_shear, s_bulk=r.s_bulk, s3=r.s3, s_h=r.s_h)
    st = M.init_state(lat, mdl, wl.rho_or_phi)
    for n in range(steps):
        st = M.step(lat, mdl, st, force=vel_at(n))
    phi, _ = M.moments(lat, mdl, st, force=vel_at(steps))
    return phi, wl.rho_or_phi.sum()


def _uniform(card, shape, u):
    u = np.asarray(u, dtype=np.float64)
    return np.broadcast_to(u.reshape((card.d,) + (1,) * card.d), (card.d,) + tuple(shape)).copy()


@pytest.mark.parametrize("card", [W.Q53_RECT, W.Q33_CUBIC], ids=lambda c: c.kind)
def test_cde_3d_gaussian_hill(card):
    N, steps, D0 = 24, 36, 0.3 * card.cs2
    adv = (0.02, -0.015, 0.01)
    shape = (N, N, N)
    phi, m0 = _cde_run(card, shape, steps, lambda n: _uniform(card, shape, adv), D0, N / 8.0)
    ref = hill_closed_form(card, shape, steps, D0, [adv[a] * steps for a in range(3)], N / 8.0)
    assert np.abs(phi - ref).max() / ref.max() < 5e-2
    assert abs(phi.sum() - m0) / m0 < 1e-12


def _rotating_error(N, steps, U=0.04, omega=None, D0=0.1):
    """2D CDE with the uniform rotating velocity u(t) = U (cos wt, sin wt):
    the hill's centre moves by (U/w)(sin wt, 1 - cos wt)."""
    card = W.Q13_SQUARE
    shape = (N, N)
    w = omega if omega is not None else 2 * np.pi / steps
    vel = lambda n: _uniform(card, shape, (U * np.cos(w * n), U * np.sin(w * n)))  # noqa: E731
    phi, m0 = _cde_run(card, shape, steps, vel, D0, N / 16.0)
    # the scheme samples u at the start of each step: the discrete path is the
    # sum of u(n), which is what the closed form's centre must follow
    path = np.array([sum(U * np.cos(w * n) for n in range(steps)), sum(U * np.sin(w * n) for n in range(steps))])
    ref = hill_closed_form(card, shape, steps, D0, path, N / 16.0)
    return np.abs(phi - ref).max() / ref.max(), abs(phi.sum() - m0) / m0


def test_cde_time_dependent_velocity():
    """A velocity that turns in time (one full turn over the run): the closed
    form with the summed path, kept mass, second-order convergence."""
    e64, dm = _rotating_error(64, 120)
    e32, _ = _rotating_error(32, 30)
    assert dm < 1e-12
    assert e64 < 1.5e-2
    assert 3.0 < e32 / e64 < 5.5
