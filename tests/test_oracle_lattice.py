"""Pins of the oracle's lattices against what the paper prints and fixes.

Every expected value here is either copied from the paper (tests/golden/),
a closed form printed in the paper, or a condition the paper states
(eqs. Cont1-5 / new11); none is produced by the oracle itself.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import lattice as L
from paper_2512_16230_amd import workloads as W

CARDS = [W.Q25_RECT, W.Q13_SQUARE, W.Q53_RECT, W.Q33_CUBIC, W.Q21_RECT, W.Q21K_RECT, W.Q45_RECT] + W.Q17_CASES


def card_lattice(card):
    return L.make_lattice(card.kind, card.c, card.cs2, card.free)


def _expr(s):
    return float(eval(s, {"__builtins__": {}}, {"sqrt": math.sqrt}))


@pytest.fixture(scope="module")
def vsets(golden_dir):
    with open(os.path.join(golden_dir, "velocity_sets.json")) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def q17(golden_dir):
    with open(os.path.join(golden_dir, "d2q17_weights.json")) as fh:
        return json.load(fh)


Q25_GROUP_INDEX = {"w0": 0, "w1": 1, "w2": 2, "w5": 5, "w9": 9, "w10": 10, "w13": 13, "w17": 17, "w18": 18,
                   "w21": 21}


def q17_lattice(q17, case):
    """rD2Q25 weights from eq. (WeightQ25) with the free weights of a printed
    D2Q17 case (square, c = 1), then the zero-weight velocities removed."""
    data = q17["cases"][str(case)]
    gmap = q17["rD2Q25_group_of"][str(case)]
    cs2 = _expr(data["cs2"])
    q25 = {g25: _expr(data[g]) for g, g25 in gmap.items()}
    free = (q25.get("w13", 0.0), q25.get("w17", 0.0), q25.get("w17", 0.0), q25.get("w21", 0.0))
    w = L.weights_rd2q25((1.0, 1.0), cs2, free)
    return data, gmap, cs2, w


# --------------------------------------------------------------------------
# velocity sets
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["rD2Q25", "rD2Q13", "rD3Q53", "rD3Q33", "D2Q21K"])
def test_velocity_sets_match_printed(vsets, kind):
    e = L.velocity_set(kind)
    assert e.tolist() == vsets[kind]["e"]
    # symmetric: -e_j is in the set for every e_j (Sec. V, below eq. new0)
    s = set(map(tuple, e.tolist()))
    assert all(tuple(-v for v in t) in s for t in s)
    assert len(s) == len(e)


@pytest.mark.parametrize("case", [1, 2, 3, 4, 5])
def test_d2q17_case_lattices_match_printed(vsets, q17, case):
    """The oracle's D2Q17 case lattices: printed velocity order, and the
    printed weights from the case card's free weights."""
    assert L.velocity_set("rD2Q17-%d" % case).tolist() == vsets["D2Q17-%d" % case]["e"]
    card = W.Q17_CASES[case - 1]
    lat = L.make_lattice(card.kind, card.c, card.cs2, card.free)
    data = q17["cases"][str(case)]
    tol = 1e-14 if data["exact"] else 5e-7
    assert abs(card.cs2 - _expr(data["cs2"])) < 1e-15
    groups = ["rest"] + [g for g in q17["groups"][1:] for _ in range(4)]
    assert np.abs(lat.w - np.array([_expr(data[g]) for g in groups])).max() < tol
    if case != 5:   # case 5 drops only groups whose weights are free (zero)
        with pytest.raises(ValueError):
            L.make_lattice(card.kind, card.c, card.cs2 * 1.01, card.free)


@pytest.mark.parametrize("case", [1, 2, 3, 4, 5])
def test_d2q17_cases_are_rd2q25_subgroups(vsets, q17, case):
    """App. C D2Q17 cases: the rD2Q25 solver with the case's free weights
    gives the printed remaining weights, and zero on the velocities the case
    drops (so the case is a subgroup lattice as stated in Sec. V)."""
    data, gmap, cs2, w = q17_lattice(q17, case)
    tol = 1e-14 if data["exact"] else 5e-7
    assert abs(w[0] - _expr(data["rest"])) < tol
    for g, g25 in gmap.items():
        assert abs(w[Q25_GROUP_INDEX[g25]] - _expr(data[g])) < tol, (g, g25)
    lat = L.subgroup(L.custom_lattice("rD2Q25", (1, 1), cs2, L.velocity_set("rD2Q25"), w), tol=1e-12)
    assert lat.b == 17
    assert set(map(tuple, lat.e.tolist())) == set(map(tuple, vsets["D2Q17-%d" % case]["e"]))


def test_d2q17_case2_as_printed_is_not_normalised(q17):
    """The printed case-2 denominators (162000, 648000) break sum w = 1."""
    data = q17["cases"]["2"]
    w0, w1, w5 = (_expr(data[k]) for k in ("rest", "g1", "g5"))
    w9p = (295 - 92 * math.sqrt(10)) / 162000
    w13p = (130 - 41 * math.sqrt(10)) / 648000
    assert abs(w0 + 4 * (w1 + w5 + w9p + w13p) - 1) > 5e-4
    w9, w13 = _expr(data["g9"]), _expr(data["g13"])
    assert abs(w0 + 4 * (w1 + w5 + w9 + w13) - 1) < 1e-14


# --------------------------------------------------------------------------
# weight conditions, eq. (Cont1-5) / (new11), by brute-force velocity sums
# --------------------------------------------------------------------------

def _check_conditions(lat, tol, sixth_square=False):
    d, cs2 = lat.d, lat.cs2
    D = lambda *ax: L.velocity_moment(lat, ax)  # noqa: E731
    assert abs(lat.w.sum() - 1) < tol
    for a in range(d):
        assert abs(D(a)) < tol
        assert abs(D(a, a) - cs2) < tol
        assert abs(D(a, a, a, a) - 3 * cs2 ** 2) < tol
        for b in range(d):
            if b != a:
                assert abs(D(a, b)) < tol
                assert abs(D(a, a, b, b) - cs2 ** 2) < tol
                assert abs(D(a, a, b)) < tol
                if sixth_square:
                    assert abs(D(a, a, a, a, b, b) - 3 * cs2 ** 3) < tol
    if d == 3:
        assert abs(D(0, 0, 1, 1, 2, 2) - cs2 ** 3) < tol


@pytest.mark.parametrize("card", CARDS, ids=lambda c: c.kind)
def test_card_weights_satisfy_conditions(card):
    lat = card_lattice(card)
    assert np.all(lat.w > 0)
    _check_conditions(lat, 1e-13)


@pytest.mark.parametrize("case", [1, 2, 3, 4])
def test_d2q17_exact_cases_satisfy_sixth_order(q17, case):
    data, _, cs2, w = q17_lattice(q17, case)
    lat = L.custom_lattice("q", (1, 1), cs2, L.velocity_set("rD2Q25"), w)
    _check_conditions(lat, 1e-13, sixth_square=True)


def test_q13_closed_form_equals_q25_with_zero_free_weights():
    """eq. (Q13lattice) closed form vs eq. (WeightQ25) with w13=w17=w18=w21=0
    on a rectangular lattice (inside 1/3 < d0a, d01 + d02 < 4/3)."""
    c, cs2 = (1.5, 1.0), 0.8
    w13 = L.weights_rd2q13(c, cs2)
    w25 = L.weights_rd2q25(c, cs2, (0, 0, 0, 0))
    assert np.allclose(w25[:13], w13, atol=1e-15, rtol=0)
    assert np.all(w25[13:] == 0)
    lat = L.custom_lattice("q13", c, cs2, L.velocity_set("rD2Q13"), w13)
    _check_conditions(lat, 1e-14)


def test_remark4_square_q25_sixth_order():
    """Remark 4: on a square rD2Q25, w13 = (d0^2 (3 d0 - 1) - 2592 w21)/192
    makes eq. (WCondQ25f) hold, i.e. Delta6_aaaabb = 3 cs^6."""
    cs2 = 1.0
    d0 = cs2
    w21 = 2e-4
    w13 = (d0 ** 2 * (3 * d0 - 1) - 2592 * w21) / 192
    w = L.weights_rd2q25((1, 1), cs2, (w13, 3e-3, 3e-3, w21))
    lat = L.custom_lattice("q25sq", (1, 1), cs2, L.velocity_set("rD2Q25"), w)
    _check_conditions(lat, 1e-13, sixth_square=True)
    # and it fails for another w13 (the relation is not automatic)
    w = L.weights_rd2q25((1, 1), cs2, (w13 + 1e-3, 3e-3, 3e-3, w21))
    lat = L.custom_lattice("q25sq", (1, 1), cs2, L.velocity_set("rD2Q25"), w)
    with pytest.raises(AssertionError):
        _check_conditions(lat, 1e-13, sixth_square=True)


def test_rd3q53_paper_family_weights():
    """App. D printed rD3Q53 family: w33 = d01 d02 (3 d01 - 1)/192 - 2 w45, ...
    satisfies eq. (new11a-d, f) (with d0a = cs^2/c_a^2, cube)."""
    c, cs2, w45 = (1.0, 1.0, 1.0), 0.6, 1e-4
    d1 = d2 = d3 = cs2
    free = (d1 * d2 * (3 * d1 - 1) / 192 - 2 * w45, d1 * d3 * (3 * d1 - 1) / 192 - 2 * w45,
            d2 * d3 * (3 * d2 - 1) / 192 - 2 * w45, w45)
    lat = L.make_lattice("rD3Q53", c, cs2, free)
    _check_conditions(lat, 1e-14)


# --------------------------------------------------------------------------
# printed transformation matrices
# --------------------------------------------------------------------------

def _load_matrix(path):
    return np.array([[int(v) for v in line.split()] for line in open(path) if not line.startswith("#")])


def _monomials(E, exps):
    return np.stack([np.prod([E[:, a] ** k for a, k in enumerate(ex)], axis=0) for ex in exps])


def test_q13_printed_transformation_matrix(golden_dir):
    c = (1.5, 1.0)
    printed = _load_matrix(os.path.join(golden_dir, "q13_transM.txt"))
    exps = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (1, 2), (2, 1), (3, 0), (0, 3), (4, 0), (2, 2), (0, 4)]
    Dm = np.array([c[0] ** a * c[1] ** b for a, b in exps])
    E = L.velocity_set("rD2Q13") * np.array(c)
    assert np.allclose(Dm[:, None] * printed, _monomials(E, exps), atol=1e-13)
    assert np.linalg.matrix_rank(printed) == 13


def test_q33_printed_transformation_matrix(golden_dir):
    """All rows but 12 (xzz) and 17 (xyz) match their monomial definitions;
    the monomial matrix has full rank, the printed one does not."""
    printed = _load_matrix(os.path.join(golden_dir, "q33_transM.txt"))
    X, Y, Z = 0, 1, 2
    def m(*ax):
        ex = [0, 0, 0]
        for a in ax:
            ex[a] += 1
        return tuple(ex)
    exps = [m(), m(X), m(Y), m(Z), m(X, X), m(Y, Y), m(Z, Z), m(X, Y), m(Z, X), m(Y, Z),
            m(X, Y, Y), m(Z, Z, X), m(X, X, Y), m(Y, Z, Z), m(Z, X, X), m(Y, Y, Z), m(X, Y, Z),
            m(X, X, X), m(Y, Y, Y), m(Z, Z, Z),
            m(X, X, Y, Y), m(Z, Z, X, X), m(Y, Y, Z, Z), m(X, X, Y, Z), m(X, Y, Y, Z), m(X, Y, Z, Z),
            m(X, X, X, X), m(Y, Y, Y, Y), m(Z, Z, Z, Z),
            m(X, X, Y, Y, Z), m(X, X, Y, Z, Z), m(X, Y, Y, Z, Z), m(X, X, Y, Y, Z, Z)]
    M = _monomials(L.velocity_set("rD3Q33").astype(float), exps)
    bad = [i for i in range(33) if not np.array_equal(M[i], printed[i])]
    assert bad == [11, 16]
    assert np.linalg.matrix_rank(M) == 33
    assert np.linalg.matrix_rank(printed) == 32


# --------------------------------------------------------------------------
# Hermite rows: weighted orthogonality and the third-order correction
# --------------------------------------------------------------------------

def _gram(lat, rows=None):
    H = lat.H(rows)
    return (H * lat.w[None, :]) @ H.T


@pytest.mark.parametrize("card", CARDS, ids=lambda c: c.kind)
def test_hermite_matrix_weighted_orthogonal(card):
    lat = card_lattice(card)
    G = _gram(lat)
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-13 * np.abs(np.diag(G)).max()
    assert len(lat.rows) == (10 if lat.d == 2 else 20)


@pytest.mark.parametrize("card", CARDS, ids=lambda c: c.kind)
def test_low_order_norms(card):
    """n_r = H_r W H_r^T for orders 0-2 follow from eq. (Cont1-5):
    1, cs^2, cs^4 (mixed), 2 d cs^4 (trace), 4 cs^4 (xx - yy)."""
    lat = card_lattice(card)
    n = dict(zip([r.name for r in lat.rows], lat.norms()))
    cs2 = lat.cs2
    assert abs(n["1"] - 1) < 1e-14
    for a in "xyz"[: lat.d]:
        assert abs(n[a] - cs2) < 1e-14
    assert abs(n["xy"] - cs2 ** 2) < 1e-13
    assert abs(n["trace"] - 2 * lat.d * cs2 ** 2) < 1e-13
    assert abs(n["xx-yy"] - 4 * cs2 ** 2) < 1e-13


def test_uncorrected_third_order_not_orthogonal_on_rectangle():
    """Sec. V below Remark 4: on a rectangular lattice H_xxx and H_xyy are
    not W-orthogonal before the correction of eq. (CorrectQ25)."""
    lat = card_lattice(W.Q25_RECT)
    cs2 = lat.cs2
    E = lat.E
    hxxx = E[:, 0] * (E[:, 0] ** 2 - 3 * cs2)
    hxyy = E[:, 0] * (E[:, 1] ** 2 - cs2)
    hyyy = E[:, 1] * (E[:, 1] ** 2 - 3 * cs2)
    hxxy = E[:, 1] * (E[:, 0] ** 2 - cs2)
    assert abs((lat.w * hxxx * hxyy).sum()) > 0.1
    assert abs((lat.w * hyyy * hxxy).sum()) > 0.01


def _paper_q53_corrections(c, cs2, free):
    """App. D closed forms a1..b3 of the rD3Q53 third-order correction."""
    w33, w37, w41, w45 = free
    d1, d2, d3 = (cs2 / ca ** 2 for ca in c)
    c1, c2, c3 = c
    a0 = 192 * w33 + 384 * w45
    b0 = 192 * w37 + 384 * w45
    c0 = 192 * w41 + 384 * w45
    a1 = c1 ** 2 / c2 ** 2 * (d1 * d2 * (1 - 3 * d1) + a0) / (d2 * d1 * (1 - d2) + a0)
    a2 = c2 ** 2 / c1 ** 2 * (d2 * d1 * (1 - 3 * d2) + a0) / (d1 * d2 * (1 - d1) + a0)
    a3 = c3 ** 2 / c1 ** 2 * (d3 * d1 * (1 - 3 * d3) + b0) / (d1 * d3 * (1 - d1) + b0)
    b1 = c1 ** 2 / c3 ** 2 * (d1 * d3 * (1 - 3 * d1) + b0) / (d3 * d1 * (1 - d3) + b0)
    b2 = c2 ** 2 / c3 ** 2 * (d2 * d3 * (1 - 3 * d2) + c0) / (d3 * d2 * (1 - d3) + c0)
    b3 = c3 ** 2 / c2 ** 2 * (d3 * d2 * (1 - 3 * d3) + c0) / (d2 * d3 * (1 - d2) + c0)
    # keys: (pure axis, mixed axis b) for the row c_a (c_b^2 - cs^2)
    return {(0, 1): a1, (0, 2): b1, (1, 0): a2, (1, 2): b2, (2, 0): a3, (2, 1): b3}


@pytest.mark.parametrize("free", [W.Q53_RECT.free, (4e-3, 1e-3, 5e-4, 1e-4)])
def test_rd3q53_correction_matches_closed_form(free):
    lat = L.make_lattice("rD3Q53", W.Q53_RECT.c, W.Q53_RECT.cs2, free)
    ref = _paper_q53_corrections(W.Q53_RECT.c, W.Q53_RECT.cs2, free)
    for k, v in ref.items():
        assert abs(lat.corrections[k] - v) < 1e-12 * max(1, abs(v)), k
    assert max(abs(v) for v in ref.values()) > 0.05


def test_rd3q53_paper_family_zeroes_some_corrections():
    c, cs2, w45 = (1.0, 1.25, 1.5), 1.0, 1e-4
    d1, d2, d3 = (cs2 / ca ** 2 for ca in c)
    free = (d1 * d2 * (3 * d1 - 1) / 192 - 2 * w45, d1 * d3 * (3 * d1 - 1) / 192 - 2 * w45,
            d2 * d3 * (3 * d2 - 1) / 192 - 2 * w45, w45)
    lat = L.make_lattice("rD3Q53", c, cs2, free)
    for k in [(0, 1), (0, 2), (1, 2)]:
        assert abs(lat.corrections[k]) < 1e-12


def test_rd3q33_correction_matches_closed_form():
    """App. D rD3Q33: H18 = x^3 - 3 cs^2 x - a1 (H11/b2 + H12/b3) etc. with
    a_a = 3 cs^2 - c_a^2 and b_a = cs^2 - c_a^2 (rectangular, not cubic)."""
    c, cs2 = (1.0, 1.1, 1.2), 0.5
    lat = L.make_lattice("rD3Q33", c, cs2)
    a = [3 * cs2 - ca ** 2 for ca in c]
    b = [cs2 - ca ** 2 for ca in c]
    ref = {(0, 1): a[0] / b[1], (0, 2): a[0] / b[2], (1, 0): a[1] / b[0], (1, 2): a[1] / b[2],
           (2, 0): a[2] / b[0], (2, 1): a[2] / b[1]}
    for k, v in ref.items():
        assert abs(lat.corrections[k] - v) < 1e-12 * max(1, abs(v)), k


def test_knight_d2q21_correction_matches_closed_form():
    """App. C knight-move D2Q21: H9 = x^3 - 3 cs^2 x - H7 a1/b1,
    H10 = y^3 - 3 cs^2 y - H8 a2/b2."""
    c, cs2, w9 = (1.2, 1.0), 0.8, 0.01
    lat = L.make_lattice("D2Q21K", c, cs2, (w9,))
    d1, d2 = cs2 / c[0] ** 2, cs2 / c[1] ** 2
    c1, c2 = c
    a1 = c1 ** 4 * c2 ** 2 * (-3 * d2 * d1 ** 2 + d2 * d1 + 48 * w9)
    b1 = c1 ** 2 * c2 ** 4 * (-d1 * d2 ** 2 + d1 * d2 + 48 * w9)
    a2 = c1 ** 2 * c2 ** 4 * (-3 * d1 * d2 ** 2 + d1 * d2 + 48 * w9)
    b2 = c1 ** 4 * c2 ** 2 * (-d2 * d1 ** 2 + d2 * d1 + 48 * w9)
    assert abs(lat.corrections[(0, 1)] - a1 / b1) < 1e-12
    assert abs(lat.corrections[(1, 0)] - a2 / b2) < 1e-12
    _check_conditions(lat, 1e-14)


def test_subgroup_rd2q21_from_zero_weight():
    """Sec. V item (i): rD2Q21 from rD2Q25 with w21 = 0; still orthogonal."""
    w = L.weights_rd2q25(W.Q25_RECT.c, W.Q25_RECT.cs2, W.Q25_RECT.free[:3] + (0.0,))
    lat = L.subgroup(L.custom_lattice("q", W.Q25_RECT.c, W.Q25_RECT.cs2, L.velocity_set("rD2Q25"), w))
    assert lat.b == 21
    G = _gram(lat)
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-13 * np.abs(np.diag(G)).max()


def test_completion_is_full_rank_and_orthogonal():
    for card in CARDS:
        lat = card_lattice(card)
        rows = L.complete_rows(lat, lat.rows)
        H = L.full_H(lat, rows)
        G = (H * lat.w) @ H.T
        assert H.shape == (lat.b, lat.b)
        assert np.abs(G - np.diag(np.diag(G))).max() < 1e-10 * np.abs(np.diag(G)).max()
        assert np.linalg.matrix_rank(H) == lat.b
