"""One time step of the Hermite-matrix MRT-LB method, in FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The state is the shifted population f_bar of eq. (2-3) (theta = gamma = 1,
full correction), or the unshifted f of the explicit three-level scheme
(theta = 1, gamma = 0), stored as an array (b, [Nz,] Ny, Nx) with x fastest.
One step is, in the paper's order:

  1. macroscopic variables, eq. (2-4-2) / (2-4-1), or eq. (2-4-0) for the
     three-level scheme; the NSE body force and mass source may be divided
     between G (F_G, S_G, corrected with lambda2, lambda1) and F (F_F, S_F);
  2. Hermite moments m = H f_bar of the rows of order <= 3 (Sec. IV);
  3. equilibrium Hermite moments m_eq from the raw moments M0..M3 the model
     prescribes: M0 = rho_bar, M1 = rho u, M2 = rho uu + p I,
     M3 = p Delta.u + M30 with M30 = rho uuu on multispeed lattices
     (eqs. M-NSEs-6a, M-NSEs-6 / M-NSEs-6-1, and the multispeed special cases
     of Sec. III), or for the NCDE M0 = phi, M1 = B = phi u,
     M2 = cs^2 D + M20 with D = Phi(phi) I and M20 = phi uu (eq. M-NCDE-6);
  4. source moments: M0F = S_F, M1F = F_F, M2F = 0 (eqs. M-NSEs-2,
     M-NSEs-5); the auxiliary moments of G are M0G = (1 - s0 lambda1/2) S_G,
     M1G = (I - lambda2 S1/2) F_G - lambda1 S10 S_G/2 and
     M2G = M2G_bar - (lambda1 S20 S_G + lambda2 S21 F_G)/2 (eqs. M-NSEs-2,
     M-NSEs-4-0) with M2G_bar = (I - S2/2)[uF + Fu + (cs^2 I - uu) S]
     (eq. M2G-1 with isothermal p and M30 = rho uuu); for the NCDE the
     auxiliary first moment of G is (I - S1/2)(d_t M1 + div M20)
     (eq. M-NCDE-6, case (1));
  5. relaxation with S in Hermite space (diagonal, except the normal
     second-order block of the standard k = 1 lattices, eq. 4-27) and the update
     m* = m - S (m - m_eq) + m_G + (I - S/2) m_F (eq. 2-3 with
     Lambda = H^-1 S H, eq. H-MRT-LB), or for the three-level scheme
     m* = m - S (m - m_eq) + m_G + m_F + (m_F(t) - m_F(t - dt))/2 (eq. 2-1);
  6. back to populations with the reduced form of eq. (H-MRT-LB-1): every row
     above third order relaxes at the single rate s_h, so
     f* = (1 - s_h) f + W sum_{r<=3} H_r^T (m*_r - (1 - s_h) m_r) / n_r;
  7. propagation f_bar_j(x + c_j dt) = f*_j(x) (eq. 2-2), periodic.

The convection-diffusion special case (3) of the NCDE section (model
"CDE"): a diffusion-type equilibrium (M0 = phi, M1 = 0, M2 = cs^2 phi I,
M3 = 0), lambda = 1, M1G = 0 and the source S_G = -u . grad(phi) with a
known velocity field u(x); the gradient comes from the non-equilibrium first
moment, grad(phi) = -S1 sum_j c_j f_j / (dt cs^2), and
phi = sum_j f_j + dt S_G / 2 (eq. M-NCDE-3-00, read with c_j in the first
sum); M0G = (1 - s0/2) S_G (eq. M-NCDE-4), so each step adds S_G to the
zeroth moment.  It recovers d_t phi + u . grad(phi) = div(K grad(phi)),
K = cs^2 (1/s1 - 1/2) dt.  The initial state is the equilibrium w_j phi.

Readings of points the paper leaves open (all listed in the design notes):
Hermite moments of F and G above their constrained orders are zero;
the equilibrium has no Hermite component above third order (eq. feq-1 with
m = 3), and none above second order for the NCDE; the NCDE time derivative
is first-order backward and the gradient is a central difference of the
previous step's phi; K = dt cs^2 (1/s1 - 1/2) (the printed (S1 - I/2) is a
typo, compare eq. ME-NCDE-3).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lattice import Lattice

NSE_INC, NSE_COMP, NCDE, CDE = "NSE_INC", "NSE_COMP", "NCDE", "CDE"


@dataclass
class Model:
    eq: str = NSE_INC
    rho0: float = 1.0
    s0: float = 1.2
    s1: float = 1.2
    s_shear: float = 1.25
    s_bulk: float = 1.2
    s3: float = 1.2
    s_h: float = 1.2
    m30: bool = True
    D0: float = 0.0          # NCDE: D(phi) = D0 (1 + D2 phi^2)
    D2: float = 0.0
    adv_u: tuple = field(default_factory=lambda: (0.0, 0.0, 0.0))
    # general NCDE (eq. M-NCDE-6): A1 dt(B_bar) = gn_bt * dt(phi) per axis
    # (B_bar = phi b_bar, gn_bt = A1 b_bar) and A2 div(D_bar) = gn_dd * grad(phi)
    # per axis (D_bar = phi I, gn_dd = diag A2)
    gn_bt: tuple = field(default_factory=lambda: (0.0, 0.0, 0.0))
    gn_dd: tuple = field(default_factory=lambda: (0.0, 0.0, 0.0))
    # NCDE source S = S_F = src_q + src_k phi (F_j with M0F = S_F, M1F = 0,
    # eqs. M-NCDE-4, M-NCDE-5) and the scheme of eq. (2-1): False = full
    # correction (theta = gamma = 1, shifted f_bar, eq. 2-3 with eq. 2-4-1),
    # True = explicit three-level scheme (theta = 1, gamma = 0: unshifted f,
    # d_t F_j by the backward difference F_j(t) - F_j(t - dt))
    src_q: float = 0.0
    src_k: float = 0.0
    three_level: bool = False
    # NSE_COMP mass source S: a number, or a field of the grid's shape
    mass_src: float = 0.0
    # NSE: the share of the body force and of the mass source that the
    # auxiliary distribution G carries, F_G = g_share F and S_G = g_share S
    # (the rest, F_F and S_F, is carried by the source distribution F; eq.
    # M-NSEs-2), and the partial-correction parameters of eqs. (2-4-0) and
    # (2-4-2).  three_level also applies to the NSE: theta = 1, gamma = 0,
    # unshifted f, F_j + (F_j(t) - F_j(t - dt)) / 2.
    g_share: float = 0.0
    lambda1: float = 1.0
    lambda2: float = 1.0
    # NSE: the form of M2G_bar.  0: the local closed form with S_bar = S and
    # d_t p + div(p u) = cs^2 S (eqs. M2Ga-1, M2G-1); 1: the gradient form,
    # eq. M2G-1 with d_t p I + div(p u I) (NSE_COMP) or eq. M2G with
    # F_bar = F - cs^2 grad(rho_bar) and S_bar = S - d_t rho_bar (NSE_INC,
    # rho = rho0), from lagged differences of the previous step's fields.
    m2g_form: int = 0

    def rate(self, group: str) -> float:
        return {"rho": self.s0, "j": self.s1, "bulk": self.s_bulk, "shear": self.s_shear,
                "third": self.s3, "high": self.s_h}[group]


def s2_normal_block(lat: Lattice, model: Model) -> np.ndarray:
    """S2 on the normal components (c_a^2 - cs^2 rows) of a standard lattice.

    eqs. (4-27), (4-27-1): S2^-1 = diag(1/s_sa) + a b^T / d with
    a_a = (1/s_ba - 1/s_sa)(c_a^2 - cs^2), b_b = 1/(c_b^2 - cs^2), and by
    eq. (4-29) with k = 1 the rates give mu = (1/s_sa - 1/2) rho (c_a^2 - cs^2)/2
    and mu_b = (1/s_ba - 1/2) rho (c_a^2 - cs^2)/d.  The model's s_shear and
    s_bulk name the target viscosities of the multispeed lattices,
    nu = cs^2 (1/s_shear - 1/2) and nu_b = (2/d) cs^2 (1/s_bulk - 1/2), so
    1/s_sa = 1/2 + 2 nu / (c_a^2 - cs^2) and 1/s_ba = 1/2 + d nu_b / (c_a^2 - cs^2).
    """
    d, cs2 = lat.d, lat.cs2
    nu = cs2 * (1.0 / model.s_shear - 0.5)
    nu_b = (2.0 / d) * cs2 * (1.0 / model.s_bulk - 0.5)
    g = np.array([lat.c[a] ** 2 - cs2 for a in range(d)])
    inv_ss = 0.5 + 2 * nu / g
    inv_sb = 0.5 + d * nu_b / g
    a_vec = (inv_sb - inv_ss) * g
    b_vec = 1.0 / g
    return np.linalg.inv(np.diag(inv_ss) + np.outer(a_vec, b_vec) / d)


def relaxation_matrix(lat: Lattice, model: Model) -> np.ndarray:
    """S on the rows of order <= 3: diagonal with the group rates, except the
    normal second-order block of a standard lattice (eq. 4-27).  The
    off-diagonal rows keep s_shear there: 1/s_ab = 1/2 + nu / cs^2 (eq. 4-29)."""
    S = np.diag([model.rate(r.group) if r.group != "normal" else 0.0 for r in lat.rows])
    idx = [i for i, r in enumerate(lat.rows) if r.group == "normal"]
    if idx:
        idx = sorted(idx, key=lambda i: lat.rows[i].axis)
        S[np.ix_(idx, idx)] = s2_normal_block(lat, model)
    return S


# --------------------------------------------------------------------------
# raw moment tensors -> Hermite moments
# --------------------------------------------------------------------------

def _raw_component(M, exp):
    idx = tuple(a for a, k in enumerate(exp) for _ in range(k))
    if len(idx) == 0:
        return M[0]
    T = M[len(idx)]
    if T is None:
        raise ValueError("raw moment of order %d not provided" % len(idx))
    return T[idx]


def hermite_from_raw(lat: Lattice, M, max_order: int) -> np.ndarray:
    """Hermite moments sum_j H_rj g_j of a distribution g whose raw moments
    sum_j g_j c_j..c_j are M = [M0, M1, M2, M3] (tensors with a trailing node
    axis); rows above ``max_order`` get zero."""
    n = np.shape(M[0])[-1]
    out = np.zeros((len(lat.rows), n))
    for r, row in enumerate(lat.rows):
        if row.order > max_order:
            continue
        for exp, coef in row.poly.items():
            out[r] += coef * _raw_component(M, exp)
    return out


def _delta_u(d, v):
    """(Delta . v)_abc = delta_ab v_c + delta_ac v_b + delta_bc v_a."""
    n = v.shape[-1]
    T = np.zeros((d, d, d, n))
    for a in range(d):
        for b in range(d):
            for c in range(d):
                T[a, b, c] = (a == b) * v[c] + (a == c) * v[b] + (b == c) * v[a]
    return T


def _uu(u):
    return np.einsum("an,bn->abn", u, u)


def _uuu(u):
    return np.einsum("an,bn,cn->abcn", u, u, u)


# --------------------------------------------------------------------------
# macroscopic variables (eq. 2-4-2 / 2-4-1)
# --------------------------------------------------------------------------

def cde_source(lat: Lattice, model: Model, f: np.ndarray, vel: np.ndarray):
    """S_G = -u . grad(phi) with grad(phi) = -s1 sum_j c_j f_j / cs^2 (CDE)."""
    grad = -model.s1 * (lat.E.T @ f) / lat.cs2
    return -(vel * grad).sum(axis=0)


def mass_field(model: Model, n: int, mass=None) -> np.ndarray:
    """The mass source S per node (n,): ``mass`` if given, else the model's
    number or field."""
    v = model.mass_src if mass is None else mass
    if np.ndim(v) == 0:
        return np.full(n, float(v))
    return np.asarray(v, dtype=np.float64).reshape(-1)


def nse_split(model: Model, force, n: int, mass=None):
    """(F_G, F_F, S_G, S_F): the body force F (d, n) or None and the mass
    source S divided between the auxiliary distribution G and the source
    distribution F, F = F_G + F_F and S = S_G + S_F (eq. M-NSEs-2)."""
    a = float(model.g_share)
    S = mass_field(model, n, mass)
    if force is None:
        return None, None, a * S, (1 - a) * S
    return a * force, (1 - a) * force, a * S, (1 - a) * S


def nse_corrections(model: Model, force, n: int):
    """The source corrections of rho and rho u: (lambda1 S_G + h S_F) / 2 and
    (lambda2 F_G + h F_F) / 2 with h = 1 for the shifted f_bar of the full
    correction (eq. 2-4-2) and h = 0 for the unshifted f of the three-level
    scheme (eq. 2-4-0); the momentum part is None without a force."""
    FG, FF, SG, SF = nse_split(model, force, n)
    h = 0.0 if model.three_level else 1.0
    r = 0.5 * (model.lambda1 * SG + h * SF)
    jc = None if force is None else 0.5 * (model.lambda2 * FG + h * FF)
    return r, jc


def macroscopic(lat: Lattice, model: Model, f: np.ndarray, force=None):
    """(rho_bar or phi, u, rho_m) from pre-collision f_bar of shape (b, n).
    For the CDE ``force`` carries the velocity field u (d, n)."""
    R0 = f.sum(axis=0)
    if model.eq == CDE:
        return R0 + 0.5 * cde_source(lat, model, f, force), force, None
    if model.eq == NCDE:
        u = np.repeat(np.asarray(model.adv_u[: lat.d], dtype=np.float64)[:, None], f.shape[1], axis=1)
        if not model.three_level:
            # eq. 2-4-1 with S_G = 0: phi = sum f_bar + S_F / 2, S_F = q + k phi
            R0 = (R0 + 0.5 * model.src_q) / (1 - 0.5 * model.src_k)
        return R0, u, None
    # eq. 2-4-2: rho = sum f_bar + (lambda1 S_G + S_F) / 2,
    # rho u = sum c f_bar + (lambda2 F_G + F_F) / 2 (eq. 2-4-0 for the
    # three-level scheme's unshifted f: no S_F, F_F terms)
    r, jc = nse_corrections(model, force, f.shape[1])
    j = lat.E.T @ f
    if jc is not None:
        j = j + jc
    R0 = R0 + r
    rho_m = np.full_like(R0, model.rho0) if model.eq == NSE_INC else R0
    return R0, j / rho_m, rho_m


def equilibrium_raw(lat: Lattice, model: Model, R0, u, rho_m):
    """Raw moments M0..M3 of f_eq prescribed by the model (None = unconstrained)."""
    d, cs2 = lat.d, lat.cs2
    I = np.eye(d)[:, :, None]
    if model.eq == CDE:
        phi = R0
        n = phi.shape[-1]
        return [phi, np.zeros((d, n)), cs2 * phi * I, np.zeros((d, d, d, n))]
    if model.eq == NCDE:
        phi = R0
        K = cs2 * (1.0 / model.s1 - 0.5)
        Phi = (model.D0 / K) * (phi + model.D2 * phi ** 3 / 3.0)
        return [phi, phi * u, cs2 * Phi * I + phi * _uu(u), None]
    p = cs2 * R0                                    # p = cs^2 rho_bar (INC) or cs^2 rho (COMP)
    M3 = p * _delta_u(d, u) if model.eq == NSE_COMP else rho_m * cs2 * _delta_u(d, u)
    if model.m30:
        M3 = M3 + rho_m * _uuu(u)
    return [R0, rho_m * u, rho_m * _uu(u) + p * I, M3]


def equilibrium_hermite(lat, model, R0, u, rho_m):
    M = equilibrium_raw(lat, model, R0, u, rho_m)
    return hermite_from_raw(lat, M, max_order=2 if model.eq == NCDE else 3)


def force_hermite(lat, n, force, mass_src=0.0):
    """Hermite moments of the source distribution F_j: M0F = S_F (mass
    source, a scalar or per node), M1F = F_F, M2F = 0 (raw moments, eqs.
    M-NSEs-2, M-NSEs-5)."""
    d = lat.d
    S = np.broadcast_to(np.asarray(mass_src, dtype=np.float64), (n,))
    if force is None and not S.any():
        return np.zeros((len(lat.rows), n))
    F = np.zeros((d, n)) if force is None else force
    M = [np.array(S), F, np.zeros((d, d, n)), None]
    return hermite_from_raw(lat, M, max_order=2)


def raw_blocks(lat: Lattice, model: Model):
    """(s0, S10, S1, S20, S21): the blocks of the collision matrix on the raw
    moments, sum_j Lambda_jk = s0, sum_j c_j Lambda_jk = S10 + S1 c_k and
    sum_j c_j c_j Lambda_jk = S20 + S21 c_k + S2 c_k c_k (Sec. III), for
    Lambda = H^-1 S H with S acting on the Hermite rows.  Summed against a
    distribution g these read sum Lambda g = s0 M0, sum c Lambda g =
    S10 M0 + S1 M1, sum cc Lambda g = S20 M0 + S21 M1 + S2 M2, so each block
    is the raw response of the relaxation to a distribution with a single
    unit raw moment: M0 = 1 gives s0, S10, S20; M1 = e_c gives column c of
    S1 and S21."""
    d = lat.d
    S = relaxation_matrix(lat, model)
    E = lat.E

    def response(M0, M1):
        m = hermite_from_raw(lat, [np.array([M0]), np.asarray(M1, dtype=np.float64).reshape(d, 1),
                                   np.zeros((d, d, 1)), None], max_order=2)
        g = populations_from_hermite(lat, S @ m)[:, 0]
        return g.sum(), E.T @ g, np.einsum("ja,jb,j->ab", E, E, g)

    s0, S10, S20 = response(1.0, np.zeros(d))
    S1 = np.zeros((d, d))
    S21 = np.zeros((d, d, d))
    for c in range(d):
        e = np.zeros(d)
        e[c] = 1.0
        _, S1[:, c], S21[:, :, c] = response(0.0, e)
    return s0, S10, S1, S20, S21


def g_route_hermite(lat: Lattice, model: Model, force, n: int):
    """Hermite moments of the part of G that carries S_G and F_G: raw
    M0G = (1 - s0 lambda1 / 2) S_G and M1G = (I - lambda2 S1 / 2) F_G
    - lambda1 S10 S_G / 2 (eq. M-NSEs-2), and the second-moment share
    -(lambda1 S20 S_G + lambda2 S21 F_G) / 2 by which M2G differs from the
    prescribed M2G_bar of ``aux_hermite`` (eq. M-NSEs-4-0)."""
    d = lat.d
    FG, _, SG, _ = nse_split(model, force, n)
    if FG is None:
        FG = np.zeros((d, n))
    s0, S10, S1, S20, S21 = raw_blocks(lat, model)
    l1, l2 = model.lambda1, model.lambda2
    M0 = (1 - 0.5 * s0 * l1) * SG
    M1 = FG - 0.5 * l2 * (S1 @ FG) - 0.5 * l1 * np.outer(S10, SG)
    M2 = -0.5 * (l1 * S20[:, :, None] * SG + l2 * np.einsum("abc,cn->abn", S21, FG))
    return hermite_from_raw(lat, [M0, M1, M2, None], max_order=2)


def m2g_gradients(lat: Lattice, model: Model, R0, j, prev):
    """The lagged differences of the gradient form of M2G_bar on the grid:
    R0 (grid) and j (d, grid) are this step's rho (rho_bar) and rho_m u,
    ``prev`` the previous step's pair (the first step uses this step's).
    NSE_COMP, isothermal p = cs^2 rho: {"div": d_t p + div(p u)} with the
    backward difference cs^2 (rho^n - rho^{n-1}) and the central difference
    of cs^2 j^{n-1}; NSE_INC: {"gr": grad(rho_bar^{n-1}) (d, n),
    "dt": rho_bar^n - rho_bar^{n-1}} (n,).  Central differences along axis a
    divide by 2 c_a (the spacing is c_a dt)."""
    d = lat.d
    r_prev, j_prev = prev
    if model.eq == NSE_COMP:
        div = (R0 - r_prev) + sum(_central(lat, j_prev[a], a) for a in range(d))
        return {"div": lat.cs2 * div.reshape(-1)}
    gr = np.stack([_central(lat, r_prev, a).reshape(-1) for a in range(d)])
    return {"gr": gr, "dt": (R0 - r_prev).reshape(-1)}


def _central(lat: Lattice, X, a: int):
    """Central difference of the grid field X along physical axis a (the
    array axis from the end; spacing c_a dt)."""
    ax = np.ndim(X) - 1 - a
    return (np.roll(X, -1, axis=ax) - np.roll(X, 1, axis=ax)) / (2 * lat.c[a])


def aux_hermite(lat, model, S, u, force, extra=None, cross=None, grad=None, mass=None):
    """Hermite moments of the auxiliary distribution G; S is the relaxation
    matrix on the rows of order <= 3.

    NSE: M2G = (I - S2/2) T with, for the local closed form,
    T = uF + Fu + (cs^2 I - uu) S_m (eqs. M2Ga-1, M2G-1), S_m the mass source
    (``mass`` per node, else the model's); for the gradient form (``grad``
    from m2g_gradients): NSE_COMP T = uF + Fu - uu S_m + (d_t p + div(p u)) I
    (eq. M2G-1, k = 0, M30 = rho uuu), NSE_INC T = u F_bar + F_bar u
    + cs^2 S_m I - uu S_bar (eq. M2G, p = cs^2 rho_bar, k = 0).
    NCDE (eq. M-NCDE-6): M1G = (I - S1/2) B - S1 X with
    B = d_t(phi u) + div(phi uu) supplied in ``extra`` and
    X = A1 d_t(B_bar) + A2 div(D_bar) in ``cross`` (general NCDE; None = 0).
    """
    n = u.shape[1]
    d = lat.d
    G = np.eye(len(lat.rows)) - 0.5 * S
    if model.eq == NCDE:
        out = np.zeros((len(lat.rows), n))
        if extra is not None:
            out += G @ hermite_from_raw(lat, [np.zeros(n), extra, None, None], max_order=1)
        if cross is not None:
            out -= S @ hermite_from_raw(lat, [np.zeros(n), cross, None, None], max_order=1)
        return out
    Sm = mass_field(model, n, mass)
    if force is None and not Sm.any() and grad is None:
        return np.zeros((len(lat.rows), n))
    F = np.zeros((d, n)) if force is None else force
    I = np.eye(d)[:, :, None]
    uu = np.einsum("an,bn->abn", u, u)
    if grad is None:
        # (cs^2 I - uu) S: eq. M2G-1 with S_bar = S, where the isothermal
        # d_t p I + div(p u I) = cs^2 (d_t rho + div(rho u)) I = cs^2 S I
        T = np.einsum("an,bn->abn", u, F) + np.einsum("an,bn->abn", F, u) + Sm * (lat.cs2 * I - uu)
    elif model.eq == NSE_COMP:
        T = np.einsum("an,bn->abn", u, F) + np.einsum("an,bn->abn", F, u) - Sm * uu + grad["div"] * I
    else:
        Fb = F - lat.cs2 * grad["gr"]
        Sb = Sm - grad["dt"]
        T = np.einsum("an,bn->abn", u, Fb) + np.einsum("an,bn->abn", Fb, u) + lat.cs2 * Sm * I - Sb * uu
    M = [np.zeros(n), np.zeros((d, n)), T, None]
    mg = hermite_from_raw(lat, M, max_order=2)
    mg[[r.order != 2 for r in lat.rows]] = 0.0
    return G @ mg


def populations_from_hermite(lat: Lattice, m: np.ndarray) -> np.ndarray:
    """g = W sum_r H_r^T m_r / n_r (eq. geq), for moments of the low rows."""
    H = lat.H()
    n = lat.norms()
    return (lat.w[:, None] * H.T) @ (m / n[:, None])


# --------------------------------------------------------------------------
# NCDE helper: B^n = u [ (phi^n - phi^{n-1}) / dt + u . grad_h phi^{n-1} ]
# --------------------------------------------------------------------------

def ncde_cross(lat: Lattice, model: Model, phi_grid: np.ndarray, phi_prev_grid: np.ndarray):
    """X^n = A1 d_t(B_bar) + A2 div(D_bar) of the general NCDE (eq. M-NCDE-6)
    with B_bar = phi b_bar and D_bar = phi I: per axis a,
    X_a = gn_bt_a (phi^n - phi^{n-1}) / dt + gn_dd_a d_a phi^{n-1}, the same
    backward time difference and central space difference of the previous
    step's phi as B^n; None when both coefficient vectors vanish."""
    d = lat.d
    bt = np.asarray(model.gn_bt[:d], dtype=np.float64)
    dd = np.asarray(model.gn_dd[:d], dtype=np.float64)
    if not (bt.any() or dd.any()):
        return None
    nd = phi_grid.ndim
    X = np.zeros((d,) + phi_grid.shape)
    for a in range(d):
        axis = nd - 1 - a
        grad = (np.roll(phi_prev_grid, -1, axis=axis) - np.roll(phi_prev_grid, 1, axis=axis)) / (2 * lat.c[a])
        X[a] = bt[a] * (phi_grid - phi_prev_grid) + dd[a] * grad
    return X.reshape(d, -1)


def ncde_B(lat: Lattice, model: Model, phi_grid: np.ndarray, phi_prev_grid: np.ndarray):
    d = lat.d
    u = np.asarray(model.adv_u[:d], dtype=np.float64)
    nd = phi_grid.ndim
    adv = np.zeros_like(phi_prev_grid)
    for a in range(d):
        axis = nd - 1 - a                       # x is the last axis
        grad = (np.roll(phi_prev_grid, -1, axis=axis) - np.roll(phi_prev_grid, 1, axis=axis)) / (2 * lat.c[a])
        adv += u[a] * grad
    scal = (phi_grid - phi_prev_grid) + adv
    return u[:, None] * scal.reshape(1, -1)


# --------------------------------------------------------------------------
# one step
# --------------------------------------------------------------------------

@dataclass
class State:
    f: np.ndarray                 # (b, *grid) pre-collision f_bar
    phi_prev: np.ndarray = None   # NCDE only: phi of the previous step
    force_prev: np.ndarray = None  # NSE three-level: the previous step's force (None: the current one)
    mass_prev: np.ndarray = None   # NSE three-level: the previous step's mass source per node
    hist: tuple = None             # NSE gradient form of M2G_bar: the previous step's (rho, rho_m u)


def ncde_source_hermite(lat: Lattice, model: Model, phi):
    """Hermite moments of the NCDE source distribution: M0F = S_F = q + k phi,
    M1F = 0 (eq. M-NCDE-5), nothing above."""
    mF = np.zeros((len(lat.rows), np.size(phi)))
    mF[[r.order == 0 for r in lat.rows]] = model.src_q + model.src_k * np.ravel(phi)
    return mF


def collide(lat: Lattice, model: Model, f: np.ndarray, force=None, ncde_b=None, ncde_x=None, phi_prev=None,
            force_prev=None, mass_prev=None, grad=None):
    """Post-collision populations f* (b, n) from pre-collision f_bar (b, n).

    ``ncde_b`` and ``ncde_x`` are the NCDE fields B^n and X^n (d, n) of the
    auxiliary first moment and ``phi_prev`` the previous step's phi (the
    three-level scheme's F(t - dt)); ``force_prev`` is the NSE three-level
    scheme's force at t - dt (None: the current force); for the CDE
    ``force`` is the velocity field (d, n); ``mass_prev`` is the mass source
    at t - dt (three-level scheme) and ``grad`` the lagged differences of
    the gradient form of M2G_bar (m2g_gradients)."""
    n = f.shape[1]
    S = relaxation_matrix(lat, model)
    R0, u, rho_m = macroscopic(lat, model, f, force)
    m = lat.H() @ f
    meq = equilibrium_hermite(lat, model, R0, u, rho_m)
    if model.eq == CDE:
        # M0G = (1 - s0/2) S_G on the zeroth row, nothing else
        mF = np.zeros_like(m)
        mG = np.zeros_like(m)
        mG[[r.order == 0 for r in lat.rows]] = (1 - 0.5 * model.s0) * cde_source(lat, model, f, force)
        mstar = m - S @ (m - meq) + mG
        return (1 - model.s_h) * f + populations_from_hermite(lat, mstar - (1 - model.s_h) * m)
    mG = aux_hermite(lat, model, S, u, force, extra=ncde_b, cross=ncde_x, grad=grad)
    if model.eq == NCDE:
        mF = ncde_source_hermite(lat, model, R0)
    else:
        _, FF, _, SF = nse_split(model, force, n)
        mF = force_hermite(lat, n, FF, SF)
        if model.g_share:
            mG = mG + g_route_hermite(lat, model, force, n)
    if model.three_level:
        # eq. 2-1 with theta = 1, gamma = 0: f - Lambda f_ne + G + F + (F(t) - F(t - dt)) / 2
        if model.eq == NCDE:
            mFp = ncde_source_hermite(lat, model, R0 if phi_prev is None else phi_prev)
        else:
            _, FFp, _, SFp = nse_split(model, force if force_prev is None else force_prev, n, mass_prev)
            mFp = force_hermite(lat, n, FFp, SFp)
        mstar = m - S @ (m - meq) + mG + mF + 0.5 * (mF - mFp)
    else:
        mstar = m - S @ (m - meq) + mG + (np.eye(len(lat.rows)) - 0.5 * S) @ mF
    return (1 - model.s_h) * f + populations_from_hermite(lat, mstar - (1 - model.s_h) * m)


def stream(lat: Lattice, fstar_grid: np.ndarray) -> np.ndarray:
    out = np.empty_like(fstar_grid)
    nd = fstar_grid.ndim - 1
    for j in range(lat.b):
        shifts = tuple(int(lat.e[j, a]) for a in range(lat.d))
        axes = tuple(nd - 1 - a for a in range(lat.d))   # x -> last axis
        out[j] = np.roll(fstar_grid[j], shifts, axis=axes)
    return out


def step(lat: Lattice, model: Model, st: State, force=None) -> State:
    grid = st.f.shape[1:]
    f = st.f.reshape(lat.b, -1)
    extra = cross = prev = None
    phi = None
    if model.eq == NCDE:
        phi = macroscopic(lat, model, f)[0].reshape(grid)
        extra = ncde_B(lat, model, phi, st.phi_prev)
        cross = ncde_cross(lat, model, phi, st.phi_prev)
        prev = st.phi_prev.reshape(-1)
    F = None if force is None else force.reshape(lat.d, -1)
    Fp = None if st.force_prev is None else st.force_prev.reshape(lat.d, -1)
    nse = model.eq in (NSE_INC, NSE_COMP)
    grad = hist = None
    if nse and model.m2g_form:
        R0, u, rho_m = macroscopic(lat, model, f, F)
        hist = (R0.reshape(grid), (rho_m * u).reshape((lat.d,) + grid))
        grad = m2g_gradients(lat, model, hist[0], hist[1], hist if st.hist is None else st.hist)
    fstar = collide(lat, model, f, F, extra, cross, prev, force_prev=Fp, mass_prev=st.mass_prev, grad=grad)
    three = nse and model.three_level
    keep = None if force is None or not three else np.array(force, dtype=np.float64)
    mkeep = mass_field(model, f.shape[1]).copy() if three else None
    return State(stream(lat, fstar.reshape(st.f.shape)), phi, keep, mkeep, hist)


def run(lat, model, st: State, steps: int, force=None) -> State:
    for _ in range(steps):
        st = step(lat, model, st, force)
    return st


# --------------------------------------------------------------------------
# initialisation and read-out
# --------------------------------------------------------------------------

def init_state(lat: Lattice, model: Model, rho_or_phi: np.ndarray, u=None, force=None) -> State:
    """f_bar(x, 0) = f_eq(rho, u) - dt/2 F (NSE) or f_eq(phi) (NCDE, CDE).

    For the NSE the subtracted distribution has the raw moments of the
    corrections of eq. (2-4-2), [(lambda1 S_G + h S_F), (lambda2 F_G + h F_F),
    0] / 2 (h = 0 for the three-level scheme), so that rho and u read back
    as given; with F_G = S_G = 0 and h = 1 it is F_j / 2."""
    grid = rho_or_phi.shape
    R0 = rho_or_phi.reshape(-1).astype(np.float64)
    n = R0.size
    if model.eq == CDE:
        meq = equilibrium_hermite(lat, model, R0, None, None)
        f = populations_from_hermite(lat, meq)
        return State(f.reshape((lat.b,) + grid), None)
    if model.eq == NCDE:
        uu = np.repeat(np.asarray(model.adv_u[: lat.d], dtype=np.float64)[:, None], n, axis=1)
        meq = equilibrium_hermite(lat, model, R0, uu, None)
        f = populations_from_hermite(lat, meq)
        if not model.three_level:
            # f_bar = f_eq - dt F / 2 with the source distribution F
            f = f - 0.5 * populations_from_hermite(lat, ncde_source_hermite(lat, model, R0))
        return State(f.reshape((lat.b,) + grid), rho_or_phi.astype(np.float64).copy())
    uv = u.reshape(lat.d, -1).astype(np.float64)
    rho_m = np.full(n, model.rho0) if model.eq == NSE_INC else R0
    meq = equilibrium_hermite(lat, model, R0, uv, rho_m)
    f = populations_from_hermite(lat, meq)
    F = None if force is None else force.reshape(lat.d, -1).astype(np.float64)
    r, jc = nse_corrections(model, F, n)
    if jc is not None or r.any():
        jc = np.zeros((lat.d, n)) if jc is None else jc
        f = f - populations_from_hermite(lat, hermite_from_raw(lat, [r, jc, np.zeros((lat.d, lat.d, n)), None], 2))
    hist = None
    if model.m2g_form:
        # the history before t = 0 from the continuity equation:
        # rho^{-1} = rho^0 - dt (S - div j^0), j^{-1} = j^0, so that the first
        # step's lagged d_t rho + div j equals S
        j0 = (rho_m * uv).reshape((lat.d,) + grid)
        div = sum(_central(lat, j0[a], a) for a in range(lat.d))
        r_prev = R0.reshape(grid) - mass_field(model, n).reshape(grid) + div
        hist = (r_prev, j0)
    return State(f.reshape((lat.b,) + grid), None, hist=hist)


def moments(lat: Lattice, model: Model, st: State, force=None):
    """(rho_bar or phi, u) on the grid at the current time."""
    grid = st.f.shape[1:]
    f = st.f.reshape(lat.b, -1)
    F = None if force is None else force.reshape(lat.d, -1)
    R0, u, _ = macroscopic(lat, model, f, F)
    return R0.reshape(grid), u.reshape((lat.d,) + grid)


def conserved(lat: Lattice, model: Model, st: State, force=None):
    f = st.f.reshape(lat.b, -1)
    mass = f.sum()
    mom = lat.E.T @ f.sum(axis=1)
    if model.eq in (NSE_INC, NSE_COMP):
        F = None if force is None else force.reshape(lat.d, -1)
        r, jc = nse_corrections(model, F, f.shape[1])
        mass = mass + r.sum()
        if jc is not None:
            mom = mom + jc.sum(axis=1)
    return float(mass), mom
