"""Brute-force formulation of the same method, for tiny grids.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Differs from ``model`` on purpose, so that each pins the other:
  * the collision is done in velocity space with an explicit b x b matrix
    Lambda = H^-1 S H (eq. H-MRT-LB), where H is the Hermite basis completed
    to b rows and H^-1 is a numerical matrix inverse (not W H^T N^-1);
  * equilibrium, source and auxiliary distributions are vectors in velocity
    space obtained as H^-1 applied to their Hermite moments (eqs. geq, feq);
  * the update is eq. (2-3) written literally:
        f*_j = f_j - Lambda_jk (f_k - f_eq_k) + G_j + (delta_jk - Lambda_jk/2) F_k;
  * macroscopic sums and propagation are explicit loops over nodes and
    populations (eq. 2-2).
"""

from __future__ import annotations

import itertools

import numpy as np

from . import model as M
from .lattice import Lattice, complete_rows, full_H


class NaiveStepper:
    def __init__(self, lat: Lattice, mdl: M.Model):
        self.lat, self.mdl = lat, mdl
        rows = complete_rows(lat, lat.rows)
        self.Hf = full_H(lat, rows)
        S_low = M.relaxation_matrix(lat, mdl)
        nlow = len(lat.rows)
        S = np.diag(np.full(lat.b, mdl.s_h))
        S[:nlow, :nlow] = S_low
        self.Hinv = np.linalg.inv(self.Hf)
        self.Lam = self.Hinv @ S @ self.Hf
        self.nlow = nlow
        self.S_low = S_low

    def _velocity_space(self, m_low):
        full = np.zeros(self.lat.b)
        full[: self.nlow] = m_low
        return self.Hinv @ full

    def step(self, st: M.State, force=None) -> M.State:
        lat, mdl = self.lat, self.mdl
        b, d = lat.b, lat.d
        grid = st.f.shape[1:]
        E = lat.E
        fstar = np.empty_like(st.f)
        phi_grid = None
        Bfield = None
        two_level_src = mdl.eq == M.NCDE and not mdl.three_level
        if mdl.eq == M.NCDE:
            phi_grid = np.zeros(grid)
            for x in itertools.product(*[range(n) for n in grid]):
                phi_grid[x] = sum(st.f[(j,) + x] for j in range(b))
                if two_level_src:
                    # phi = sum f_bar + (q + k phi) / 2 solved for phi
                    phi_grid[x] = (phi_grid[x] + 0.5 * mdl.src_q) / (1 - 0.5 * mdl.src_k)
            Bfield = M.ncde_B(lat, mdl, phi_grid, st.phi_prev).reshape((d,) + grid)
            Xfield = M.ncde_cross(lat, mdl, phi_grid, st.phi_prev)
            if Xfield is not None:
                Xfield = Xfield.reshape((d,) + grid)
        for x in itertools.product(*[range(n) for n in grid]):
            f = np.array([st.f[(j,) + x] for j in range(b)])
            F = None if force is None else np.array([force[(a,) + x] for a in range(d)])
            rho = 0.0
            mom = np.zeros(d)
            for j in range(b):
                rho += f[j]
                mom += E[j] * f[j]
            if mdl.eq == M.NCDE:
                u = np.asarray(mdl.adv_u[:d], dtype=np.float64)
                rho_m = None
                rho = phi_grid[x]
            else:
                if F is not None:
                    mom = mom + 0.5 * F
                rho = rho + 0.5 * mdl.mass_src      # rho = sum f_bar + S / 2
                rho_m = mdl.rho0 if mdl.eq == M.NSE_INC else rho
                u = mom / rho_m
            R0 = np.array([rho])
            uv = u[:, None]
            rm = None if rho_m is None else np.array([rho_m])
            feq = self._velocity_space(M.equilibrium_hermite(lat, mdl, R0, uv, rm)[:, 0])
            if mdl.eq == M.NCDE:
                Bx = np.array([Bfield[(a,) + x] for a in range(d)])[:, None]
                Xx = None if Xfield is None else np.array([Xfield[(a,) + x] for a in range(d)])[:, None]
                G = self._velocity_space(M.aux_hermite(lat, mdl, self.S_low, uv, None, extra=Bx, cross=Xx)[:, 0])
                Fv = self._velocity_space(M.ncde_source_hermite(lat, mdl, R0)[:, 0])
                if mdl.three_level:
                    Fp = self._velocity_space(M.ncde_source_hermite(lat, mdl, st.phi_prev[x])[:, 0])
                    # eq. 2-1, theta = 1, gamma = 0: F + (F(t) - F(t - dt)) / 2, no (I - Lambda/2)
                    out = f - self.Lam @ (f - feq) + G + Fv + 0.5 * (Fv - Fp)
                    for j in range(b):
                        fstar[(j,) + x] = out[j]
                    continue
            else:
                Fa = None if F is None else F[:, None]
                G = self._velocity_space(M.aux_hermite(lat, mdl, self.S_low, uv, Fa)[:, 0])
                Fv = (np.zeros(b) if F is None and not mdl.mass_src
                      else self._velocity_space(M.force_hermite(lat, 1, Fa, mdl.mass_src)[:, 0]))
            out = f - self.Lam @ (f - feq) + G + (np.eye(b) - 0.5 * self.Lam) @ Fv
            for j in range(b):
                fstar[(j,) + x] = out[j]
        # propagation, one population and one node at a time
        new = np.empty_like(fstar)
        for j in range(b):
            for x in itertools.product(*[range(n) for n in grid]):
                # grid index order is (.., y, x): the physical axis a lives at
                # array axis len(grid) - 1 - a
                tgt = list(x)
                for a in range(d):
                    ax = len(grid) - 1 - a
                    tgt[ax] = (x[ax] + int(lat.e[j, a])) % grid[ax]
                new[(j,) + tuple(tgt)] = fstar[(j,) + x]
        return M.State(new, phi_grid)
