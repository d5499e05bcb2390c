"""The pins must catch plausible mistakes in the oracle.

Each test plants one mistake in an oracle function (monkeypatch, CPU only,
undone after the test) and checks that a pin which holds for the correct
oracle fails: a dropped term, a wrong sign, a wrong weighting, swapped
rates, a reversed direction, a wrong constant.  Nothing here touches the GPU
library.
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import model as M
from paper_2512_16230_amd import workloads as W

import test_oracle_collision as TC
import test_oracle_dynamics as TD
import test_oracle_lattice as TL


def _pin_fails(pin, *args):
    with pytest.raises((AssertionError, np.linalg.LinAlgError, ValueError)):
        pin(*args)


def test_pins_hold_unmutated():
    TC.test_equilibrium_moments_nse(W.Q25_RECT, M.NSE_COMP)
    TC.test_collision_is_bgk_with_guo_forcing_when_rates_equal()
    TL.test_hermite_matrix_weighted_orthogonal(W.Q25_RECT)
    TL.test_card_weights_satisfy_conditions(W.Q25_RECT)
    TC.test_vectorised_step_equals_brute_force(W.Q25_RECT, M.NSE_INC, (4, 3))


def test_dropped_m30_is_caught(monkeypatch):
    monkeypatch.setattr(M, "_uuu", lambda u: np.zeros((u.shape[0],) * 3 + (u.shape[1],)))
    _pin_fails(TC.test_equilibrium_moments_nse, W.Q25_RECT, M.NSE_COMP)


def test_wrong_viscous_third_moment_is_caught(monkeypatch):
    orig = M._delta_u
    monkeypatch.setattr(M, "_delta_u", lambda d, v: 0.9 * orig(d, v))
    _pin_fails(TC.test_equilibrium_moments_nse, W.Q53_RECT, M.NSE_COMP)


def test_wrong_sign_of_m2g_is_caught(monkeypatch):
    orig = M.aux_hermite
    monkeypatch.setattr(M, "aux_hermite", lambda *a, **k: -orig(*a, **k))
    _pin_fails(TC.test_collision_is_bgk_with_guo_forcing_when_rates_equal)


def test_missing_half_force_in_u_is_caught(monkeypatch):
    orig = M.macroscopic
    monkeypatch.setattr(M, "macroscopic", lambda lat, model, f, force=None: orig(lat, model, f, None))
    _pin_fails(TC.test_collision_is_bgk_with_guo_forcing_when_rates_equal)


def test_unweighted_correction_is_caught(monkeypatch):
    monkeypatch.setattr(L, "_inner", lambda lat, p, q: float((L.poly_eval(p, lat.E) * L.poly_eval(q, lat.E)).sum()))
    _pin_fails(TL.test_hermite_matrix_weighted_orthogonal, W.Q25_RECT)


def test_wrong_weight_formula_is_caught(monkeypatch):
    orig = L.weights_rd2q25

    def bad(c, cs2, free):
        w = orig(c, cs2, free).copy()
        w[5:9] += 1e-3          # the (1, 1) group
        w[0] -= 4e-3            # still sums to one
        return w
    monkeypatch.setattr(L, "weights_rd2q25", bad)
    _pin_fails(TL.test_card_weights_satisfy_conditions, W.Q25_RECT)


def test_reversed_streaming_is_caught(monkeypatch):
    def backwards(lat, fstar_grid):
        out = np.empty_like(fstar_grid)
        nd = fstar_grid.ndim - 1
        for j in range(lat.b):
            shifts = tuple(-int(lat.e[j, a]) for a in range(lat.d))
            out[j] = np.roll(fstar_grid[j], shifts, axis=tuple(nd - 1 - a for a in range(lat.d)))
        return out
    monkeypatch.setattr(M, "stream", backwards)
    _pin_fails(TC.test_vectorised_step_equals_brute_force, W.Q25_RECT, M.NSE_INC, (4, 3))


def test_swapped_shear_and_bulk_rates_are_caught(monkeypatch):
    orig = M.Model.rate
    swap = {"shear": "bulk", "bulk": "shear"}
    monkeypatch.setattr(M.Model, "rate", lambda self, g: orig(self, swap.get(g, g)))
    _pin_fails(TD.test_taylor_green_2d_decay_and_convergence)


def test_wrong_ncde_diffusion_constant_is_caught(monkeypatch):
    orig = M.equilibrium_raw

    def bad(lat, model, R0, u, rho_m):
        out = orig(lat, model, R0, u, rho_m)
        if model.eq == M.NCDE:
            out[2] = 1.1 * out[2]      # Phi off by 10%: D = K Phi' wrong
        return out
    monkeypatch.setattr(M, "equilibrium_raw", bad)
    _pin_fails(TD.test_gaussian_hill_linear_diffusion)


def test_wrong_cde_gradient_is_caught(monkeypatch):
    orig = M.cde_source
    monkeypatch.setattr(M, "cde_source", lambda *a: 0.5 * orig(*a))
    _pin_fails(TD.test_cde_gaussian_hill_closed_form)
