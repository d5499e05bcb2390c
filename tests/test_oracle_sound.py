"""Acoustic pins of the multispeed lattices: the trace of the normal
second-order Hermite rows relaxes at s_bulk.

A small standing sound wave in the isothermal compressible model is damped
at (k^2/2)[2 nu (1 - 1/d) + nu_b] and travels at cs, with
nu = cs^2 (1/s_shear - 1/2) dt and nu_b = (2/d) cs^2 (1/s_bulk - 1/2) dt
(eq. 4-29 with k = 0, Sec. III; the longitudinal viscosity of the
recovered Navier-Stokes equations).  Divergence-free flows (Taylor-Green,
shear waves) cannot see nu_b; a compressional wave can, along every axis of
the rectangular rD2Q25 (dx/dy = 1.5) and rD3Q53 (1 : 1.25 : 1.5).  The bulk
and shear rates are chosen far apart (0.9 against 1.25), so relaxing the
trace at the shear rate moves the damping by about 30%.
"""

import numpy as np
import pytest
from scipy.optimize import curve_fit

from oracle import lattice as L
from oracle import model as M
from paper_2512_16230_amd import workloads as W

S_SHEAR, S_BULK = 1.25, 0.9


def sound_wave(card, axis, n, eps=1e-4):
    """Grid shape, wavenumber, coordinate and initial density of a standing
    wave along ``axis`` (one cell thick in the other directions)."""
    d = len(card.c)
    shape = [1] * d
    shape[d - 1 - axis] = n
    shape = tuple(shape)
    k = 2 * np.pi / (n * card.c[axis])
    x = W.axis_coords(card, shape, axis) * np.ones(shape)
    return shape, k, x, 1 + eps * np.cos(k * x)


def damping_and_speed(card, axis, n=48, steps=240, eps=1e-4, s_shear=S_SHEAR, s_bulk=S_BULK):
    """(fitted damping / predicted, fitted frequency / (cs k))."""
    lat = L.make_lattice(card.kind, card.c, card.cs2, card.free)
    d = lat.d
    mdl = M.Model(eq=M.NSE_COMP, s_shear=s_shear, s_bulk=s_bulk, s3=1.1, s_h=1.1)
    shape, k, x, rho = sound_wave(card, axis, n, eps)
    st = M.init_state(lat, mdl, rho, np.zeros((d,) + shape))
    amp = []
    for _ in range(steps):
        r, _ = M.moments(lat, mdl, st)
        amp.append(((r - 1) * np.cos(k * x)).sum() / (0.5 * n * eps))
        st = M.step(lat, mdl, st)
    t = np.arange(steps, dtype=np.float64)
    fit = lambda t, A, g, om, ph: A * np.exp(-g * t) * np.cos(om * t + ph)  # noqa: E731
    p, _ = curve_fit(fit, t, np.array(amp), p0=(1.0, 1e-3, np.sqrt(lat.cs2) * k, 0.0))
    nu = lat.cs2 * (1 / s_shear - 0.5)
    nu_b = (2 / d) * lat.cs2 * (1 / s_bulk - 0.5)
    return p[1] / (0.5 * k * k * (2 * nu * (1 - 1 / d) + nu_b)), p[2] / (np.sqrt(lat.cs2) * k)


CASES = [(W.Q25_RECT, 0), (W.Q25_RECT, 1), (W.Q53_RECT, 0), (W.Q53_RECT, 2)]


@pytest.mark.parametrize("card,axis", CASES, ids=["rD2Q25-x", "rD2Q25-y", "rD3Q53-x", "rD3Q53-z"])
def test_sound_damping_sets_the_bulk_viscosity(card, axis):
    ratio, speed = damping_and_speed(card, axis)
    assert abs(ratio - 1) < 0.005
    assert abs(speed - 1) < 0.005


def test_bulk_and_shear_rates_enter_separately():
    """Two bulk rates at one shear rate: both damping rates match the closed
    form, which they could not if the trace row ignored s_bulk."""
    for sb in (0.8, 1.6):
        ratio, _ = damping_and_speed(W.Q25_RECT, 0, s_bulk=sb)
        assert abs(ratio - 1) < 0.005
