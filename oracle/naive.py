"""Brute-force formulation of the same method, for tiny grids.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Differs from ``model`` on purpose, so that each pins the other:
  * the collision is done in velocity space with an explicit b x b matrix
    Lambda = H^-1 S H (eq. H-MRT-LB), where H is the Hermite basis completed
    to b rows and H^-1 is a numerical matrix inverse (not W H^T N^-1);
  * equilibrium, source and auxiliary distributions are vectors in velocity
    space obtained as H^-1 applied to their Hermite moments (eqs. geq, feq);
  * the update is eq. (2-3) written literally:
        f*_j = f_j - Lambda_jk (f_k - f_eq_k) + G_j + (delta_jk - Lambda_jk/2) F_k,
    or eq. (2-1) with theta = 1, gamma = 0 for the three-level scheme;
  * the raw-moment blocks s0, S10, S1, S20, S21 that the NSE's partial
    correction uses (eqs. M-NSEs-2, M-NSEs-4-0) are read off the columns of
    Lambda by their defining sums: the rest velocity's column gives s0,
    S10, S20, and the columns of +-c_a e_a give S1 and S21 by differences;
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
        self._read_blocks()

    def _read_blocks(self):
        """sum_j Lambda_jk = s0, sum_j c_j Lambda_jk = S10 + S1 c_k and
        sum_j c_j c_j Lambda_jk = S20 + S21 c_k + S2 c_k c_k, evaluated on
        the columns k of the rest velocity and of the unit steps +-e_a."""
        lat, E, Lam = self.lat, self.lat.E, self.Lam
        d = lat.d
        col1 = E.T @ Lam                                   # (d, b): sum_j c_j Lambda_jk
        col2 = np.einsum("ja,jb,jk->abk", E, E, Lam)       # (d, d, b)
        rest = [k for k in range(lat.b) if not lat.e[k].any()][0]
        self.s0 = float(Lam[:, rest].sum())
        self.S10 = col1[:, rest].copy()
        self.S20 = col2[:, :, rest].copy()
        self.S1 = np.zeros((d, d))
        self.S21 = np.zeros((d, d, d))
        for a in range(d):
            unit = np.zeros(d, dtype=int)
            unit[a] = 1
            kp = [k for k in range(lat.b) if (lat.e[k] == unit).all()][0]
            km = [k for k in range(lat.b) if (lat.e[k] == -unit).all()][0]
            span = 2 * lat.c[a]
            self.S1[:, a] = (col1[:, kp] - col1[:, km]) / span
            self.S21[:, :, a] = (col2[:, :, kp] - col2[:, :, km]) / span

    def _raw_to_velocity(self, M0, M1, M2):
        """The velocity-space distribution whose raw moments of order <= 2
        are M0, M1, M2 and whose Hermite moments above order 2 vanish."""
        Mr = [np.array([M0]), np.asarray(M1, dtype=np.float64).reshape(-1, 1),
              np.asarray(M2, dtype=np.float64).reshape(self.lat.d, self.lat.d, 1), None]
        return self._velocity_space(M.hermite_from_raw(self.lat, Mr, max_order=2)[:, 0])

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
        nse = mdl.eq in (M.NSE_INC, M.NSE_COMP)
        Sgrid = None
        if nse:
            ms = mdl.mass_src
            Sgrid = np.full(grid, float(ms)) if np.ndim(ms) == 0 else np.asarray(ms, dtype=np.float64).reshape(grid)
        Rg = Jg = prev = None
        if nse and mdl.m2g_form:
            # the gradient form of M2G_bar: every node's rho and rho_m u first
            Rg, Jg = np.zeros(grid), np.zeros((d,) + grid)
            for x in itertools.product(*[range(n) for n in grid]):
                F = None if force is None else np.array([force[(a,) + x] for a in range(d)])
                rho, u, rho_m = self._nse_macro(st.f, x, F, Sgrid[x])
                Rg[x] = rho
                for a in range(d):
                    Jg[(a,) + x] = rho_m * u[a]
            prev = (Rg, Jg) if st.hist is None else st.hist
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
                share = mdl.g_share
                Ftot = np.zeros(d) if F is None else F
                Sx = Sgrid[x]
                FG, FF = share * Ftot, (1 - share) * Ftot
                SG, SF = share * Sx, (1 - share) * Sx
                rho, u, rho_m = self._nse_macro(st.f, x, F, Sx)
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
                if mdl.m2g_form:
                    G = self._m2g_gradient_form(st.f.shape[1:], x, u, Ftot, Sx, Rg, prev)
                else:
                    G = self._velocity_space(M.aux_hermite(lat, mdl, self.S_low, uv, Fa, mass=np.array([Sx]))[:, 0])
                if share:
                    # the S_G, F_G part of G: M0G, M1G (eq. M-NSEs-2) and the
                    # share of M2G beside M2G_bar (eq. M-NSEs-4-0)
                    l1, l2 = mdl.lambda1, mdl.lambda2
                    M0G = (1 - 0.5 * self.s0 * l1) * SG
                    M1G = FG - 0.5 * l2 * (self.S1 @ FG) - 0.5 * l1 * self.S10 * SG
                    M2G = -0.5 * (l1 * self.S20 * SG + l2 * np.einsum("abc,c->ab", self.S21, FG))
                    G = G + self._raw_to_velocity(M0G, M1G, M2G)
                Fv = self._raw_to_velocity(SF, FF, np.zeros((d, d)))
                if mdl.three_level:
                    Fp = Ftot if st.force_prev is None else np.array([st.force_prev[(a,) + x] for a in range(d)])
                    SFp = SF if st.mass_prev is None else (1 - share) * np.asarray(st.mass_prev).reshape(grid)[x]
                    Fvp = self._raw_to_velocity(SFp, (1 - share) * Fp, np.zeros((d, d)))
                    # eq. 2-1, theta = 1, gamma = 0
                    out = f - self.Lam @ (f - feq) + G + Fv + 0.5 * (Fv - Fvp)
                    for j in range(b):
                        fstar[(j,) + x] = out[j]
                    continue
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
        keep = mkeep = None
        if nse and mdl.three_level:
            keep = None if force is None else np.array(force, dtype=np.float64)
            mkeep = Sgrid.reshape(-1).copy()
        return M.State(new, phi_grid, keep, mkeep, None if Rg is None else (Rg, Jg))

    def _nse_macro(self, fgrid, x, F, Sx):
        """(rho, u, rho_m) of one node: F = F_G + F_F, S = S_G + S_F, rho and
        rho u by eq. 2-4-2 (eq. 2-4-0 for the three-level scheme's unshifted
        f: no F_F, S_F terms)."""
        lat, mdl = self.lat, self.mdl
        d = lat.d
        rho = 0.0
        mom = np.zeros(d)
        for j in range(lat.b):
            rho += fgrid[(j,) + x]
            mom += lat.E[j] * fgrid[(j,) + x]
        share, h = mdl.g_share, (0.0 if mdl.three_level else 1.0)
        Ftot = np.zeros(d) if F is None else F
        mom = mom + 0.5 * (mdl.lambda2 * share * Ftot + h * (1 - share) * Ftot)
        rho = rho + 0.5 * (mdl.lambda1 * share * Sx + h * (1 - share) * Sx)
        rho_m = mdl.rho0 if mdl.eq == M.NSE_INC else rho
        return rho, mom / rho_m, rho_m

    def _m2g_gradient_form(self, grid, x, u, F, Sx, Rg, prev):
        """G of the gradient form of M2G_bar at node x, T built one component
        at a time: NSE_COMP T_ab = u_a F_b + F_a u_b - S u_a u_b
        + delta_ab (d_t p + div(p u)) with p = cs^2 rho, the backward time
        difference and the central space difference of the previous step's
        rho u; NSE_INC T_ab = u_a Fb_b + Fb_a u_b + cs^2 S delta_ab - Sb u_a u_b
        with Fb = F - cs^2 grad(rho_bar^{n-1}) and Sb = S - (rho_bar^n -
        rho_bar^{n-1}).  M2G_bar = (I - S2/2) T on the second-order rows."""
        lat, mdl = self.lat, self.mdl
        d, cs2 = lat.d, lat.cs2
        rp, jp = prev

        def nb(a, step):
            t = list(x)
            ax = len(grid) - 1 - a
            t[ax] = (x[ax] + step) % grid[ax]
            return tuple(t)

        T = np.zeros((d, d))
        if mdl.eq == M.NSE_COMP:
            div = Rg[x] - rp[x]
            for a in range(d):
                div += (jp[(a,) + nb(a, 1)] - jp[(a,) + nb(a, -1)]) / (2 * lat.c[a])
            div *= cs2
            for a in range(d):
                for b in range(d):
                    T[a, b] = u[a] * F[b] + F[a] * u[b] - Sx * u[a] * u[b] + (div if a == b else 0.0)
        else:
            Fb = np.array([F[a] - cs2 * (rp[nb(a, 1)] - rp[nb(a, -1)]) / (2 * lat.c[a]) for a in range(d)])
            Sb = Sx - (Rg[x] - rp[x])
            for a in range(d):
                for b in range(d):
                    T[a, b] = u[a] * Fb[b] + Fb[a] * u[b] + (cs2 * Sx if a == b else 0.0) - Sb * u[a] * u[b]
        mg = M.hermite_from_raw(lat, [np.zeros(1), np.zeros((d, 1)), T[:, :, None], None], max_order=2)[:, 0]
        mg[[r.order != 2 for r in lat.rows]] = 0.0
        return self._velocity_space((np.eye(self.nlow) - 0.5 * self.S_low) @ mg)
