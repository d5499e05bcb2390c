"""Lattices of the oracle: velocity sets, weights and Hermite rows, in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper references (arXiv 2512.16230):
  * velocity moments Delta^(k) ............... Sec. V, eq. (new0)
  * weighted-orthogonality conditions ........ Sec. V, eqs. (Cont1-5), (new11)
  * rD2Q25 velocities / weights .............. Sec. V, eqs. (3-1), (3-1-2), (WeightQ25)
  * rD2Q13 velocities / closed-form weights .. Sec. V, eq. (Q13lattice)
  * third-order correction ................... Sec. V, eqs. (CorrectQ25), (CorrectQ25-1)
  * D2Q17 cases 1-5, knight-move D2Q21 ....... App. C
  * rD3Q53 / rD3Q33 velocities and weights ... App. D
  * Hermite rows H0..H3 ...................... Sec. V (definition above eq. (new5)),
                                               App. C/D lists of H rows
  * standard D2Q9 / D3Q27 (k = 1) ............. Sec. IV, eqs. (4-27), (4-27-1), and the
                                               standard-lattice case of Sec. IV-B

Everything here is the plain definition: weights from the printed formulas,
Hermite rows as polynomials in the physical velocity, the third-order
correction as a W-weighted Gram-Schmidt projection.  The trace/deviator
rotation of the normal second-order rows is the reading that lets a diagonal
S carry separate bulk and shear rates (rows stay W-orthogonal because all
c_s,alpha are equal, Remark 2).
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field
import numpy as np

# --------------------------------------------------------------------------
# velocity sets (integer multiples e_j; physical c_j = diag(c) e_j)
# --------------------------------------------------------------------------

_D2Q9_RING = [(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def _rd2q25():
    # eq. (3-1): rest, then layers s = 1, 2, 3 of the D2Q9 ring in that order
    return [(0, 0)] + [(s * a, s * b) for s in (1, 2, 3) for (a, b) in _D2Q9_RING]


def _rd2q13():
    # eq. (Q13lattice)
    return [(0, 0)] + _D2Q9_RING + [(2, 0), (0, 2), (-2, 0), (0, -2)]


# App. D, printed velocity matrix of rD3Q53 (first block: D3Q27 in the
# paper's column order; second block: twice the non-rest columns).
_D3Q27_X = [0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1]
_D3Q27_Y = [0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, -1, 1, 1, -1]
_D3Q27_Z = [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1]


def _rd3q53():
    base = list(zip(_D3Q27_X, _D3Q27_Y, _D3Q27_Z))
    return base + [(2 * a, 2 * b, 2 * c) for (a, b, c) in base[1:]]


def _rd3q33():
    # App. D, printed velocity matrix of rD3Q33: D3Q27 then (+-2,0,0),(0,+-2,0),(0,0,+-2)
    base = list(zip(_D3Q27_X, _D3Q27_Y, _D3Q27_Z))
    return base + [(2, 0, 0), (-2, 0, 0), (0, 2, 0), (0, -2, 0), (0, 0, 2), (0, 0, -2)]


# App. C, knight-move D2Q21 (not a subgroup of rD2Q25)
_KNIGHT21 = [(0, 0)] + _D2Q9_RING + [(2, 1), (1, 2), (-1, 2), (-2, 1), (-2, -1), (-1, -2), (1, -2), (2, -1),
                                     (3, 0), (0, 3), (-3, 0), (0, -3)]


# App. C, the printed velocity matrices of the D2Q17 cases 1-5 (square,
# c = 1 there): each keeps the rest velocity and four of the rD2Q25 groups.
_Q17_GROUPS = {
    1: ["ring1", "diag1", "diag2", "axis3"],
    2: ["ring1", "diag1", "axis3", "diag3"],
    3: ["diag1", "axis2", "axis3", "diag3"],
    4: ["diag1", "diag2", "axis3", "diag3"],
    5: ["ring1", "diag1", "axis2", "diag2"],
}


def _q17(case):
    axis = [(1, 0), (0, 1), (-1, 0), (0, -1)]
    diag = [(1, 1), (-1, 1), (-1, -1), (1, -1)]
    groups = {"ring1": axis, "diag1": diag, "axis2": [(2 * a, 2 * b) for a, b in axis],
              "diag2": [(2 * a, 2 * b) for a, b in diag], "axis3": [(3 * a, 3 * b) for a, b in axis],
              "diag3": [(3 * a, 3 * b) for a, b in diag]}
    return [(0, 0)] + [v for g in _Q17_GROUPS[case] for v in groups[g]]


def _d3q27():
    return list(zip(_D3Q27_X, _D3Q27_Y, _D3Q27_Z))


# Standard (single-layer) lattices: the k = 1 model of the standard-lattice
# special case, with no pure third-order rows and a non-diagonal S2 block.
STANDARD = ("D2Q9", "D3Q27")


def velocity_set(kind: str) -> np.ndarray:
    """Integer velocity multiples e_j (b x d) in the paper's column order."""
    table = {
        "rD2Q25": _rd2q25,
        "rD2Q13": _rd2q13,
        "rD3Q53": _rd3q53,
        "rD3Q33": _rd3q33,
        "D2Q21K": lambda: _KNIGHT21,
        # Sec. V item (i): rD2Q25 without its (+-3, +-3) group (w21 = 0)
        "rD2Q21": lambda: _rd2q25()[:21],
        # the rD3Q53 subgroup without its (+-2, +-2, +-2) group (w45 = 0)
        "rD3Q45": lambda: _rd3q53()[:45],
        **{"rD2Q17-%d" % k: (lambda k=k: _q17(k)) for k in range(1, 6)},
        # the first layer of rD2Q25 / rD3Q53 (eq. 3-1, App. D)
        "D2Q9": lambda: [(0, 0)] + _D2Q9_RING,
        "D3Q27": _d3q27,
    }
    return np.array(table[kind](), dtype=np.int64)


# --------------------------------------------------------------------------
# weights
# --------------------------------------------------------------------------

def _group_weights(e: np.ndarray, group_of) -> np.ndarray:
    return np.array([group_of(tuple(int(v) for v in row)) for row in e], dtype=np.float64)


def weights_rd2q25(c, cs2, free):
    """eq. (WeightQ25) with free (w13, w17, w18, w21); d0a = cs^2 / c_a^2."""
    d1, d2 = cs2 / c[0] ** 2, cs2 / c[1] ** 2
    w13, w17, w18, w21 = (float(v) for v in free)
    w5 = 0.25 * (d1 * d2 - 64 * w13 - 324 * w21)
    w9 = (d1 * (3 * d1 - 1) - 48 * w13 - 144 * w17 - 288 * w21) / 24
    w10 = (d2 * (3 * d2 - 1) - 48 * w13 - 144 * w18 - 288 * w21) / 24
    w1 = 0.5 * d1 - (2 * w5 + 4 * w9 + 8 * w13 + 9 * w17 + 18 * w21)
    w2 = 0.5 * d2 - (2 * w5 + 4 * w10 + 8 * w13 + 9 * w18 + 18 * w21)
    # eq. (3-1-2): w0 = 1 - sum_{j>0} w_j
    w0 = 1 - 2 * (w1 + w2 + w9 + w10 + w17 + w18) - 4 * (w5 + w13 + w21)

    def g(v):
        a, b = abs(v[0]), abs(v[1])
        s = max(a, b)
        if s == 0:
            return w0
        layer = {1: (w1, w2, w5), 2: (w9, w10, w13), 3: (w17, w18, w21)}[s]
        if b == 0:
            return layer[0]
        if a == 0:
            return layer[1]
        return layer[2]

    return _group_weights(velocity_set("rD2Q25"), g)


def weights_standard(e, c, cs2):
    """Standard-lattice weights: the product of one D1Q3 weight per axis,
    1 - d_a at rest and d_a / 2 at +-1, d_a = cs^2 / c_a^2.

    On the single-layer set these are the only weights that meet the
    conditions of Sec. V the lattice can meet: unit mass, Delta2 = cs^2 I and
    the mixed fourth moments Delta4_aabb = cs^4 that make the second-order
    rows W-orthogonal.  The pure fourth moments are c_a^2 cs^2, not 3 cs^4;
    the k = 1 model absorbs that difference in its S2 block (eq. 4-27-1).
    """
    d = np.array([cs2 / ca ** 2 for ca in c])
    w = np.ones(len(e))
    for j, v in enumerate(e):
        for a, t in enumerate(v):
            w[j] *= d[a] / 2 if t != 0 else 1 - d[a]
    return w


def weights_rd2q13(c, cs2):
    """Closed-form weights printed with eq. (Q13lattice)."""
    d1, d2 = cs2 / c[0] ** 2, cs2 / c[1] ** 2
    w9 = d1 * (3 * d1 - 1) / 24
    w10 = d2 * (3 * d2 - 1) / 24
    w0 = (1 - d1) * (1 - d2) + 6 * (w9 + w10)
    w1 = d1 * (1 - d2) / 2 - 4 * w9
    w2 = d2 * (1 - d1) / 2 - 4 * w10
    w5 = d1 * d2 / 4
    return np.array([w0, w1, w2, w1, w2, w5, w5, w5, w5, w9, w10, w9, w10])


def weights_rd3q53(c, cs2, free):
    """App. D rD3Q53 weights with free (w33, w37, w41, w45).

    The printed definition of d0a inverts the ratio; the weight equations
    (new11) need d0a = c_sa^2 / c_a^2 (Sec. V, below eq. (new11)).
    """
    d1, d2, d3 = (cs2 / ca ** 2 for ca in c)
    w33, w37, w41, w45 = (float(v) for v in free)
    w19 = d1 * d2 * d3 / 8 - 64 * w45
    w7 = d1 * d2 / 4 - 2 * w19 - 16 * w33 - 32 * w45
    w11 = d1 * d3 / 4 - 2 * w19 - 16 * w37 - 32 * w45
    w15 = d2 * d3 / 4 - 2 * w19 - 16 * w41 - 32 * w45
    w27 = d1 * (3 * d1 - 1) / 24 - 2 * (w33 + w37) - 4 * w45
    w28 = d2 * (3 * d2 - 1) / 24 - 2 * (w33 + w41) - 4 * w45
    w29 = d3 * (3 * d3 - 1) / 24 - 2 * (w41 + w37) - 4 * w45
    w1 = d1 / 2 - 2 * (w7 + w11) - 4 * w19 - 4 * w27 - 8 * (w33 + w37) - 16 * w45
    w2 = d2 / 2 - 2 * (w7 + w15) - 4 * w19 - 4 * w28 - 8 * (w33 + w41) - 16 * w45
    w3 = d3 / 2 - 2 * (w11 + w15) - 4 * w19 - 4 * w29 - 8 * (w41 + w37) - 16 * w45
    w0 = (1 - 2 * (w1 + w2 + w3 + w27 + w28 + w29)
          - 4 * (w7 + w11 + w15 + w33 + w37 + w41) - 8 * (w19 + w45))
    layer1 = {"x": w1, "y": w2, "z": w3, "xy": w7, "xz": w11, "yz": w15, "xyz": w19}
    layer2 = {"x": w27, "y": w28, "z": w29, "xy": w33, "xz": w37, "yz": w41, "xyz": w45}
    return _layered_3d(velocity_set("rD3Q53"), w0, layer1, layer2)


def weights_rd3q33(c, cs2):
    """App. D rD3Q33 weights (unique for a given c_s^2)."""
    d1, d2, d3 = (cs2 / ca ** 2 for ca in c)
    w19 = d1 * d2 * d3 / 8
    w7 = d1 * d2 / 4 - 2 * w19
    w11 = d1 * d3 / 4 - 2 * w19
    w15 = d2 * d3 / 4 - 2 * w19
    w27 = d1 * (3 * d1 - 1) / 24
    w28 = d2 * (3 * d2 - 1) / 24
    w29 = d3 * (3 * d3 - 1) / 24
    w1 = d1 / 2 - 2 * (w7 + w11) - 4 * w19 - 4 * w27
    w2 = d2 / 2 - 2 * (w7 + w15) - 4 * w19 - 4 * w28
    w3 = d3 / 2 - 2 * (w11 + w15) - 4 * w19 - 4 * w29
    w0 = 1 - 2 * (w1 + w2 + w3 + w27 + w28 + w29) - 4 * (w7 + w11 + w15) - 8 * w19
    layer1 = {"x": w1, "y": w2, "z": w3, "xy": w7, "xz": w11, "yz": w15, "xyz": w19}
    layer2 = {"x": w27, "y": w28, "z": w29}
    return _layered_3d(velocity_set("rD3Q33"), w0, layer1, layer2)


def _layered_3d(e, w0, layer1, layer2):
    def g(v):
        s = max(abs(t) for t in v)
        if s == 0:
            return w0
        key = "".join(ax for ax, t in zip("xyz", v) if t != 0)
        return (layer1 if s == 1 else layer2)[key]

    return _group_weights(e, g)


def weights_knight21(c, cs2, w9):
    """App. C knight-move D2Q21 weights with free w9."""
    d1, d2 = cs2 / c[0] ** 2, cs2 / c[1] ** 2
    w5 = d1 * d2 / 4 - 8 * w9
    w17 = (d1 * (3 * d1 - 1) - 48 * w9) / 144
    w18 = (d2 * (3 * d2 - 1) - 48 * w9) / 144
    w1 = d1 / 2 - 2 * w5 - 10 * w9 - 9 * w17
    w2 = d2 / 2 - 2 * w5 - 10 * w9 - 9 * w18
    w0 = 1 - 2 * (w1 + w2 + 2 * w5 + 4 * w9 + w17 + w18)
    return np.array([w0, w1, w2, w1, w2] + [w5] * 4 + [w9] * 8 + [w17, w18, w17, w18])


# --------------------------------------------------------------------------
# Hermite rows as polynomials in the physical velocity
# --------------------------------------------------------------------------

Poly = dict  # exponent tuple -> coefficient


def _mono(d, *axes):
    exp = [0] * d
    for a in axes:
        exp[a] += 1
    return tuple(exp)


def poly_add(*terms):
    """Sum of (coef, poly) pairs."""
    out: dict = {}
    for coef, p in terms:
        for k, v in p.items():
            out[k] = out.get(k, 0.0) + coef * v
    return {k: v for k, v in out.items() if v != 0.0}


def poly_eval(p: Poly, E: np.ndarray) -> np.ndarray:
    """Evaluate a polynomial on the rows of E (b x d physical velocities)."""
    out = np.zeros(E.shape[0])
    for exp, coef in p.items():
        term = np.full(E.shape[0], coef)
        for a, k in enumerate(exp):
            if k:
                term = term * E[:, a] ** k
        out += term
    return out


@dataclass
class Row:
    name: str
    order: int
    group: str          # relaxation group: rho, j, bulk, shear, normal, third, high
    poly: Poly
    axis: int = -1      # normal second-order component rows: their axis


@dataclass
class Lattice:
    kind: str
    c: tuple
    cs2: float
    e: np.ndarray               # integer multiples, b x d
    w: np.ndarray               # weights, b
    rows: list = field(default_factory=list)      # Hermite rows of order 0..3
    corrections: dict = field(default_factory=dict)

    @property
    def d(self):
        return self.e.shape[1]

    @property
    def b(self):
        return self.e.shape[0]

    @property
    def E(self):
        return self.e * np.asarray(self.c, dtype=np.float64)[None, :]

    def H(self, rows=None):
        rows = self.rows if rows is None else rows
        return np.stack([poly_eval(r.poly, self.E) for r in rows])

    def norms(self, rows=None):
        H = self.H(rows)
        return (H * H * self.w[None, :]).sum(axis=1)


def velocity_moment(lat: Lattice, axes) -> float:
    """Delta^(k)_{i1..ik} = sum_j w_j c_{j,i1} ... c_{j,ik}   (eq. new0)."""
    E = lat.E
    prod = np.ones(lat.b)
    for a in axes:
        prod = prod * E[:, a]
    return float((lat.w * prod).sum())


def _inner(lat, p, q):
    return float((lat.w * poly_eval(p, lat.E) * poly_eval(q, lat.E)).sum())


def hermite_rows(lat: Lattice) -> tuple[list, dict]:
    """Rows H0..H3 (Sec. V) with the rectangular-lattice correction.

    Orders 0-2: H0 = 1, H1 = c, H2 = cc - Delta2 with Delta2 = cs^2 I.  The
    normal rows of H2 are rotated into a trace row and deviator rows, so a
    diagonal S separates bulk and shear rates.
    Order 3: mixed rows c_a (c_b^2 - cs^2) (a != b), c_x c_y c_z in 3D, and
    the pure rows c_a (c_a^2 - 3 cs^2) corrected by removing their W-weighted
    projection on span{c_a (c_b^2 - cs^2) : b != a} (eq. CorrectQ25 and its
    App. D analogue).  Returns (rows, correction coefficients).
    Standard lattices keep the normal component rows c_a^2 - cs^2 (their S2
    block is not diagonal, eq. 4-27) and have no pure third-order rows.
    """
    d, cs2 = lat.d, lat.cs2
    standard = lat.kind in STANDARD
    one = {_mono(d): 1.0}
    ax = "xyz"[:d]
    rows = [Row("1", 0, "rho", one)]
    for a in range(d):
        rows.append(Row(ax[a], 1, "j", {_mono(d, a): 1.0}))
    hnorm = [poly_add((1.0, {_mono(d, a, a): 1.0}), (-cs2, one)) for a in range(d)]
    if standard:
        # component rows c_a^2 - cs^2, relaxed together by the S2 block
        for a in range(d):
            rows.append(Row(ax[a] * 2, 2, "normal", hnorm[a], axis=a))
    elif d == 2:
        rows.append(Row("trace", 2, "bulk", poly_add(*[(1.0, h) for h in hnorm])))
        rows.append(Row("xx-yy", 2, "shear", poly_add((1.0, hnorm[0]), (-1.0, hnorm[1]))))
    else:
        rows.append(Row("trace", 2, "bulk", poly_add(*[(1.0, h) for h in hnorm])))
        rows.append(Row("xx-yy", 2, "shear", poly_add((1.0, hnorm[0]), (-1.0, hnorm[1]))))
        rows.append(Row("xx+yy-2zz", 2, "shear",
                        poly_add((1.0, hnorm[0]), (1.0, hnorm[1]), (-2.0, hnorm[2]))))
    for a, b in itertools.combinations(range(d), 2):
        rows.append(Row(ax[a] + ax[b], 2, "shear", {_mono(d, a, b): 1.0}))

    mixed = {}
    for a in range(d):
        for b in range(d):
            if a != b:
                mixed[(a, b)] = poly_add((1.0, {_mono(d, a, b, b): 1.0}), (-cs2, {_mono(d, a): 1.0}))
    third = []
    for a in range(d):
        for b in range(d):
            if a != b:
                third.append(Row(ax[a] + ax[b] + ax[b], 3, "third", mixed[(a, b)]))
    if d == 3:
        third.append(Row("xyz", 3, "third", {_mono(d, 0, 1, 2): 1.0}))
    corrections = {}
    if standard:
        # c_a^3 = c_a^2 c_a on a single layer: the pure rows are multiples of
        # the first-order rows and are not part of the basis
        rows += third
        return rows, corrections
    for a in range(d):
        pure = poly_add((1.0, {_mono(d, a, a, a): 1.0}), (-3 * cs2, {_mono(d, a): 1.0}))
        basis = [mixed[(a, b)] for b in range(d) if b != a]
        G = np.array([[_inner(lat, p, q) for q in basis] for p in basis])
        rhs = np.array([_inner(lat, pure, p) for p in basis])
        coef = np.linalg.solve(G, rhs)
        for b_, k in zip([b for b in range(d) if b != a], coef):
            corrections[(a, b_)] = float(k)
        corrected = poly_add((1.0, pure), *[(-k, p) for k, p in zip(coef, basis)])
        third.append(Row(ax[a] * 3, 3, "third", corrected))
    rows += third
    return rows, corrections


def complete_rows(lat: Lattice, rows: list, tol: float = 1e-9) -> list:
    """Extend rows to a W-orthogonal basis of R^b (rows of order >= 4).

    The paper leaves rows above third order to the user (App. C/D).  Greedy
    choice: monomials of increasing total degree, W-Gram-Schmidt against the
    rows kept so far, keep a monomial when its residual is non-negligible.
    """
    d = lat.d
    W = lat.w
    basis = [poly_eval(r.poly, lat.E) for r in rows]
    out = list(rows)
    deg = 4
    while len(out) < lat.b and deg < 16:
        for exp in sorted((t for t in itertools.product(range(deg + 1), repeat=d) if sum(t) == deg),
                          reverse=True):
            if len(out) == lat.b:
                break
            v = poly_eval({exp: 1.0}, lat.E)
            for bvec in basis:
                v = v - (W * v * bvec).sum() / (W * bvec * bvec).sum() * bvec
            scale = np.sqrt((W * poly_eval({exp: 1.0}, lat.E) ** 2).sum())
            if np.sqrt((W * v * v).sum()) > tol * max(scale, 1.0):
                basis.append(v)
                out.append(Row("m" + "".join(map(str, exp)), deg, "high", None))
                out[-1].values = v  # numeric row (no closed polynomial kept)
        deg += 1
    if len(out) != lat.b:
        raise ValueError("could not complete the Hermite basis")
    return out


def full_H(lat: Lattice, rows: list) -> np.ndarray:
    return np.stack([r.values if r.poly is None else poly_eval(r.poly, lat.E) for r in rows])


def make_lattice(kind: str, c=(1.0, 1.0), cs2=None, free=None) -> Lattice:
    """Build a lattice card: velocities, weights, corrected Hermite rows."""
    e = velocity_set(kind)
    c = tuple(float(v) for v in c)
    if kind == "rD2Q25":
        w = weights_rd2q25(c, cs2, free)
    elif kind == "rD2Q13":
        w = weights_rd2q13(c, cs2)
    elif kind == "rD3Q53":
        w = weights_rd3q53(c, cs2, free)
    elif kind == "rD3Q33":
        w = weights_rd3q33(c, cs2)
    elif kind == "D2Q21K":
        w = weights_knight21(c, cs2, free[0])
    elif kind == "rD2Q21":
        w = weights_rd2q25(c, cs2, tuple(free) + (0.0,))[:21]
    elif kind == "rD3Q45":
        w = weights_rd3q53(c, cs2, tuple(free) + (0.0,))[:45]
    elif kind in STANDARD:
        w = weights_standard(e, c, cs2)
    elif kind.startswith("rD2Q17-"):
        # eq. (WeightQ25) on the full rD2Q25 set; the dropped groups must vanish
        e25 = velocity_set("rD2Q25")
        w25 = weights_rd2q25(c, cs2, free)
        keep = {tuple(v) for v in e.tolist()}
        dropped = [w25[j] for j in range(len(e25)) if tuple(e25[j].tolist()) not in keep]
        if max(abs(v) for v in dropped) > 1e-12:
            raise ValueError("cs2 and the free weights do not give D2Q17 case " + kind)
        index = {tuple(v): j for j, v in enumerate(e25.tolist())}
        w = np.array([w25[index[tuple(v)]] for v in e.tolist()])
    else:
        raise ValueError(kind)
    return custom_lattice(kind, c, cs2, e, w)


def custom_lattice(kind, c, cs2, e, w) -> Lattice:
    """Lattice from an explicit velocity set and weights."""
    lat = Lattice(kind=kind, c=tuple(float(v) for v in c), cs2=float(cs2),
                  e=np.asarray(e, dtype=np.int64), w=np.asarray(w, dtype=np.float64))
    lat.rows, lat.corrections = hermite_rows(lat)
    return lat


def subgroup(lat: Lattice, tol: float = 1e-14) -> Lattice:
    """Subgroup lattice: drop the velocities whose weight is zero (Sec. V,
    items (i)-(iii) after eq. CorrectQ25: rD2Q21, rD2Q17, rD2Q13 obtained
    from rD2Q25 by zeroing weights)."""
    keep = np.abs(lat.w) > tol
    return custom_lattice(lat.kind + "-sub", lat.c, lat.cs2, lat.e[keep], lat.w[keep])
