"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds workload parameters and initial/forcing fields only; it
contains none of the lattice Boltzmann arithmetic (no weights, no Hermite
rows, no equilibria).  Every field is FP64 on the host, laid out with x
fastest: scalars (Ny, Nx) or (Nz, Ny, Nx), vectors (d, Ny, Nx) or
(d, Nz, Ny, Nx).  Positions are physical: x = i * dx_a with dx_a = c_a dt,
dt = 1.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from math import pi

import numpy as np

# ---------------------------------------------------------------------------
# lattice cards (kind, c_alpha, cs^2, free weights).  The free weights are a
# parameter choice: a point well inside the region where every weight is
# positive (analytic centre of the positivity polytope, rounded).
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class Card:
    kind: str
    c: tuple
    cs2: float
    free: tuple = ()

    @property
    def d(self):
        return len(self.c)


Q25_RECT = Card("rD2Q25", (1.5, 1.0), 1.5, (5.35e-3, 6.25e-4, 2.46e-2, 8.2e-4))
Q13_SQUARE = Card("rD2Q13", (1.0, 1.0), 0.5)
Q53_RECT = Card("rD3Q53", (1.0, 1.25, 1.5), 1.0, (6.56e-3, 2.05e-3, 3.0e-4, 2.3e-4))
Q33_CUBIC = Card("rD3Q33", (1.0, 1.0, 1.0), 0.45)
# subgroup rD2Q21 (w21 = 0) and the knight-move D2Q21 on the rD2Q25 aspect ratio
Q21_RECT = Card("rD2Q21", (1.5, 1.0), 1.5, (8.0e-3, 1.6e-3, 3.3e-2))
Q21K_RECT = Card("D2Q21K", (1.5, 1.0), 0.98, (7.0e-4,))
# App. C, D2Q17 cases 1-5 (square): the printed cs^2 and, as rD2Q25 free
# weights (w13, w17, w18, w21), the printed weights of the kept groups
_R193, _R10 = 193 ** 0.5, 10 ** 0.5
Q17_CASES = [
    Card("rD2Q17-1", (1.0, 1.0), 72 / (125 + 5 * _R193),
         ((685 - 49 * _R193) / 54000, (1445 - 101 * _R193) / 162000, (1445 - 101 * _R193) / 162000, 0.0)),
    Card("rD2Q17-2", (1.0, 1.0), 3 / (5 + _R10),
         (0.0, (295 - 92 * _R10) / 16200, (295 - 92 * _R10) / 16200, (130 - 41 * _R10) / 64800)),
    Card("rD2Q17-3", (1.0, 1.0), 3 / 4, (0.0, 1 / 1440, 1 / 1440, 5 / 18432)),
    Card("rD2Q17-4", (1.0, 1.0), 3 / 2, (9 / 640, 1 / 36, 1 / 36, 23 / 11520)),
    Card("rD2Q17-5", (1.0, 1.0), 0.3740845, (0.0000891, 0.0, 0.0, 0.0)),
]
# subgroup rD3Q45 (w45 = 0) at the rD3Q53 aspect ratio
Q45_RECT = Card("rD3Q45", (1.0, 1.25, 1.5), 0.86, (4.3e-3, 4.8e-4, 4.3e-4))
# standard single-layer lattices (k = 1 model, non-diagonal S2 block) on
# the same aspect ratios; every weight is positive for cs^2 < min c_a^2
Q9_RECT = Card("D2Q9", (1.5, 1.0), 0.5)
Q9_SQUARE = Card("D2Q9", (1.0, 1.0), 1 / 3)
Q27_RECT = Card("D3Q27", (1.0, 1.25, 1.5), 0.6)


@dataclass
class Rates:
    s0: float = 1.2
    s1: float = 1.2
    s_shear: float = 1.25
    s_bulk: float = 1.2
    s3: float = 1.2
    s_h: float = 1.2


def rates_tau(tau_shear: float, other: float = 1.2) -> Rates:
    """Shear rate 1/tau, every other diagonal entry of S equal to ``other``."""
    return Rates(other, other, 1.0 / tau_shear, other, other, other)


# ---------------------------------------------------------------------------
# fields
# ---------------------------------------------------------------------------

def axis_coords(card: Card, shape, a):
    """Physical coordinates along axis a (x = 0), shaped to broadcast."""
    d = card.d
    n = shape[d - 1 - a]                   # x is the last array axis
    sh = [1] * d
    sh[d - 1 - a] = n
    return (np.arange(n, dtype=np.float64) * card.c[a]).reshape(sh)


def grid_coords(card: Card, shape):
    """Physical coordinates, one array per axis, broadcast to ``shape``."""
    return [np.broadcast_to(axis_coords(card, shape, a), shape) for a in range(card.d)]


def taylor_green_2d(card: Card, shape, U0, rho0=1.0, t=0.0, nu=0.0):
    """Incompressible 2D Taylor-Green vortex on a periodic rectangle.

    kx = 2 pi / Lx, ky = 2 pi / Ly (Lx = Nx dx, Ly = Ny dy);
    u = -U0 sqrt(ky/kx) cos(kx x) sin(ky y) F, v = U0 sqrt(kx/ky) sin(kx x) cos(ky y) F,
    p = -(rho0 U0^2 / 4) [ (ky/kx) cos(2 kx x) + (kx/ky) cos(2 ky y) ] F^2,
    F = exp(-nu (kx^2 + ky^2) t).  Returns (p, u) with u of shape (2, Ny, Nx).
    Separable factors are evaluated on the axes and combined by broadcasting.
    """
    Ny, Nx = shape
    kx = 2 * pi / (Nx * card.c[0])
    ky = 2 * pi / (Ny * card.c[1])
    x = axis_coords(card, shape, 0)
    y = axis_coords(card, shape, 1)
    F = np.exp(-nu * (kx * kx + ky * ky) * t)
    u = (-U0 * np.sqrt(ky / kx) * F) * np.cos(kx * x) * np.sin(ky * y)
    v = (U0 * np.sqrt(kx / ky) * F) * np.sin(kx * x) * np.cos(ky * y)
    p = (-(rho0 * U0 * U0 / 4) * F * F) * ((ky / kx) * np.cos(2 * kx * x) + (kx / ky) * np.cos(2 * ky * y))
    return p, np.stack([u, v])


def taylor_green_3d(card: Card, shape, U0, drho=1e-2):
    """3D Taylor-Green start: u = U0 sin(kx x) cos(ky y) cos(kz z),
    v = -U0 (kx/ky) cos(kx x) sin(ky y) cos(kz z), w = 0 (divergence free),
    rho = 1 + drho cos(kx x) cos(ky y) cos(kz z).  Returns (rho, u (3, ...))."""
    Nz, Ny, Nx = shape
    kx = 2 * pi / (Nx * card.c[0])
    ky = 2 * pi / (Ny * card.c[1])
    kz = 2 * pi / (Nz * card.c[2])
    x, y, z = (axis_coords(card, shape, a) for a in range(3))
    cz = np.cos(kz * z)
    u = (U0 * np.sin(kx * x)) * (np.cos(ky * y) * cz)
    v = (-U0 * (kx / ky) * np.cos(kx * x)) * (np.sin(ky * y) * cz)
    w = np.zeros(shape)
    rho = 1.0 + (drho * np.cos(kx * x)) * (np.cos(ky * y) * cz)
    return rho, np.stack([u, v, w])


def gaussian_hill(card: Card, shape, amplitude=1.0, sigma0=None, center=None):
    """phi0 = A exp(-|x - x0|^2 / (2 sigma0^2)) with periodic images summed
    (images at +-1 period in each axis), sigma0 in physical units.  The
    Gaussian and its image sum factor over the axes."""
    d = card.d
    L = [shape[d - 1 - a] * card.c[a] for a in range(d)]
    if sigma0 is None:
        sigma0 = min(L) / 16.0
    if center is None:
        center = [0.5 * La for La in L]
    out = amplitude
    for a in range(d):
        xa = axis_coords(card, shape, a)
        g = sum(np.exp(-(xa - center[a] + k * L[a]) ** 2 / (2 * sigma0 ** 2)) for k in (-1, 0, 1))
        out = out * g
    return np.broadcast_to(out, shape).copy()


def sinusoidal_force(card: Card, shape, F0, seed, modes=3):
    """F(x) = F0 sum_m n_m sin(k_m . x + phase_m), n_m seeded unit vectors,
    k_m seeded integer wave vectors of the periodic box."""
    rng = np.random.default_rng(seed)
    d = card.d
    L = [shape[d - 1 - a] * card.c[a] for a in range(d)]
    F = np.zeros((d,) + tuple(shape))
    for _ in range(modes):
        n = rng.normal(size=d)
        n /= np.linalg.norm(n)
        k = rng.integers(1, 3, size=d) * rng.choice([-1, 1], size=d)
        ph = rng.uniform(0, 2 * pi)
        # sin(sum_a t_a + ph) expanded with complex exponentials per axis
        e = np.exp(1j * ph)
        for a in range(d):
            e = e * np.exp(1j * 2 * pi * k[a] / L[a] * axis_coords(card, shape, a))
        arg_sin = np.broadcast_to(e.imag, shape)
        F += F0 * n.reshape((d,) + (1,) * d) * arg_sin[None]
    return F


def flow_bounds(eq, rho_or_phi, u=None, force=None, steps=0, rho0=1.0, adv_u=(0.0, 0.0, 0.0), margin=1.5,
                cs2=None, mass_src=0.0):
    """Run-long bounds (u_bound, dev_bound) on max |u| and on max |rho - rho0|
    / rho0 (NSE) or max |phi| (NCDE, CDE), from the initial fields: ``margin``
    times the initial maxima, which bound an unforced run (decaying kinetic
    energy; maximum principle of the convection-diffusion equation), plus for
    a body force the velocity it can add in ``steps`` steps, max |F| steps /
    min rho, and (given cs2) the pressure deviation u_bound^2 / cs2 of that
    flow; a mass source S adds |S| steps / rho0 to the density bound.  (The
    library adds the NCDE equilibrium's diffusion term itself.)"""
    if eq == "NCDE":
        return margin * float(np.linalg.norm(adv_u)), margin * float(np.abs(rho_or_phi).max())
    if eq == "CDE":
        umax = float(np.sqrt((np.asarray(u) ** 2).sum(0)).max())
        return margin * umax, margin * float(np.abs(rho_or_phi).max())
    rho = np.asarray(rho_or_phi)
    umax = float(np.sqrt((np.asarray(u) ** 2).sum(0)).max()) if u is not None else 0.0
    dev = float(np.abs(rho - rho0).max()) / rho0
    if force is not None:
        umax += float(np.sqrt((np.asarray(force) ** 2).sum(0)).max()) * steps / float(rho.min())
        if cs2:
            dev += (margin * umax) ** 2 / cs2
    dev += abs(mass_src) * steps / rho0
    return margin * umax, margin * dev


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    card: Card
    eq: str                       # NSE_INC, NSE_COMP, NCDE
    shape: tuple                  # (Ny, Nx) or (Nz, Ny, Nx)
    steps: int
    rates: Rates
    rho0: float = 1.0
    rho_or_phi: np.ndarray = None
    u: np.ndarray = None
    force: np.ndarray = None
    adv_u: tuple = (0.0, 0.0, 0.0)
    D0: float = 0.0
    D2: float = 0.0
    meta: dict = field(default_factory=dict)


def tgv_small(seed=0, shape=(64, 64), steps=500):
    """rD2Q25 incompressible Taylor-Green vortex, 64 x 64, dx/dy = 1.5,
    U0 ~ U[0.01, 0.05] (seeded), rho0 = 1, tau_shear = 0.8, other rates 1.2."""
    rng = np.random.default_rng(seed)
    U0 = 0.01 + 0.04 * rng.uniform()
    card = Q25_RECT
    p, u = taylor_green_2d(card, shape, U0)
    rho_bar = 1.0 + p / card.cs2
    return Workload("tgv-rD2Q25-%dx%d" % (shape[1], shape[0]), card, "NSE_INC", shape, steps,
                    rates_tau(0.8), 1.0, rho_bar, u, meta={"U0": U0})


def tgv_large(seed=0, shape=(4096, 4096), steps=1000, sigma=1e-3, card=Q25_RECT):
    """Incompressible Taylor-Green vortex at Ma = 0.1 (U0 = 0.1 cs) plus iid
    N(0, sigma^2) per velocity component, tau_shear = 0.6 (rD2Q25 unless
    another 2D card is given)."""
    rng = np.random.default_rng(seed)
    U0 = 0.1 * np.sqrt(card.cs2)
    p, u = taylor_green_2d(card, shape, U0)
    u = u + rng.normal(0.0, sigma, size=u.shape)
    rho_bar = 1.0 + p / card.cs2
    return Workload("tgv-%s-%dx%d" % (card.kind, shape[1], shape[0]), card, "NSE_INC", shape, steps,
                    rates_tau(0.6), 1.0, rho_bar, u, meta={"U0": U0, "sigma": sigma})


def tgv3d(shape=(256, 256, 256), steps=1000, U0=0.05, drho=1e-2, card=Q53_RECT):
    """Compressible isothermal 3D Taylor-Green start on rD3Q53 (1 : 1.25 : 1.5)."""
    rho, u = taylor_green_3d(card, shape, U0, drho)
    return Workload("tgv3d-%s-%dx%dx%d" % (card.kind, shape[2], shape[1], shape[0]), card, "NSE_COMP",
                    shape, steps, rates_tau(0.8), 1.0, rho, u, meta={"U0": U0})


def ncde_hill(shape=(128, 128), steps=1000, adv_u=(0.03, -0.02), D0=0.1, D2=1.0, card=Q13_SQUARE):
    """rD2Q13 NCDE: Gaussian hill (amplitude 1, sigma0 = N/16), constant
    advection, D(phi) = D0 (1 + D2 phi^2), s1 chosen so K = D0."""
    K = D0
    s1 = 1.0 / (K / card.cs2 + 0.5)
    r = Rates(1.2, s1, 1.2, 1.2, 1.2, 1.2)
    phi = gaussian_hill(card, shape)
    return Workload("ncde-%s-%dx%d" % (card.kind, shape[1], shape[0]), card, "NCDE", shape, steps, r,
                    0.0, phi, None, adv_u=tuple(adv_u) + (0.0,) * (3 - len(adv_u)), D0=D0, D2=D2)


def shear_field(card: Card, shape, U):
    """Divergence-free velocity field u = (U sin(2 pi y / Ly), 0) on a 2D box."""
    y = axis_coords(card, shape, 1)
    Ly = shape[0] * card.c[1]
    ux = np.broadcast_to(U * np.sin(2 * pi * y / Ly), shape)
    return np.stack([ux, np.zeros(shape)])


def cde_hill(shape=(128, 128), steps=1000, u=(0.03, -0.02), D0=0.1, card=Q13_SQUARE):
    """Convection-diffusion (CDE special case of the NCDE) of a Gaussian hill
    (amplitude 1, sigma0 = N/16) in a velocity field: ``u`` is a constant
    vector or a (d, Ny, Nx) field; diffusivity D0 via s1 (K = D0)."""
    s1 = 1.0 / (D0 / card.cs2 + 0.5)
    r = Rates(1.2, s1, 1.2, 1.2, 1.2, 1.2)
    phi = gaussian_hill(card, shape)
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 1:
        u = np.broadcast_to(u.reshape((card.d,) + (1,) * card.d), (card.d,) + tuple(shape)).copy()
    return Workload("cde-%s-%dx%d" % (card.kind, shape[1], shape[0]), card, "CDE", shape, steps, r,
                    0.0, phi, u, D0=D0)


def ncde_batch_sizes(n=256, lo=128, hi=1024, seed=0):
    """Log-uniform square side lengths for a batch of NCDE solves."""
    rng = np.random.default_rng(seed)
    return [int(round(np.exp(rng.uniform(np.log(lo), np.log(hi))))) for _ in range(n)]


def ncde_batch(n=256, lo=128, hi=1024, seed=0, steps=1000):
    rng = np.random.default_rng(seed + 1)
    out = []
    for N in ncde_batch_sizes(n, lo, hi, seed):
        adv = tuple(rng.uniform(-0.05, 0.05, size=2))
        out.append(ncde_hill((N, N), steps, adv_u=adv))
    return out
