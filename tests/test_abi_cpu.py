"""CPU checks of the C-ABI library: it is built, loads, exports every
symbol declared in include/mrtlb.h, and its host-side lattice builder
(no GPU involved) agrees with the oracle's independent construction."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import lattice as OL
from paper_2512_16230_amd import _mrtlb as H
from paper_2512_16230_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mrtlb.h")).read()
    decl = r"^(?:mrtlb_status|void|int|int64_t|const char\*)\s+\**(mrtlb_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(H.LIB_PATH), "libmrtlb.so not built"
    lib = ctypes.CDLL(H.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(lib, s)]
    assert missing == []
    assert sorted(H.EXPORTED) == syms


def test_version():
    assert H.lib().mrtlb_version() >> 16 == 1


@pytest.mark.parametrize("card", [W.Q25_RECT, W.Q13_SQUARE, W.Q53_RECT, W.Q33_CUBIC, W.Q21_RECT, W.Q21K_RECT,
                                  W.Q45_RECT, W.Q9_RECT, W.Q27_RECT] + W.Q17_CASES,
                         ids=lambda c: c.kind)
def test_host_lattice_matches_oracle(card):
    q = H.Lattice(card.kind, card.c, card.cs2, card.free).query()
    lat = OL.make_lattice(card.kind, card.c, card.cs2, card.free)
    assert np.array_equal(q["e"], lat.e)
    assert np.allclose(q["w"], lat.w, rtol=0, atol=1e-15)
    Hm = q["H"]
    G = (Hm * q["w"]) @ Hm.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-13 * np.abs(np.diag(G)).max()
    assert np.allclose(np.diag(G), q["norms"], rtol=1e-14)
    # the library's component rows span the same space as the oracle's rows
    # (rotated second-order rows there), order by order
    Ho = lat.H()
    for order in range(4):
        A = Ho[[r.order == order for r in lat.rows]]
        rank_A = np.linalg.matrix_rank(A)
        idx = {0: [0], 1: list(range(1, 1 + lat.d))}
        if order >= 2:
            n2 = lat.d * (lat.d + 1) // 2
            idx[2] = list(range(1 + lat.d, 1 + lat.d + n2))
            idx[3] = list(range(1 + lat.d + n2, Hm.shape[0]))
        Bm = Hm[idx[order]]
        assert np.linalg.matrix_rank(np.vstack([A, Bm]), tol=1e-9) == rank_A == Bm.shape[0]
    if card.kind in OL.STANDARD:
        # no pure third-order rows on a single layer
        assert q["H"].shape[0] == len(lat.rows) == (8 if lat.d == 2 else 17)
        return
    # corrected pure third-order rows are identical (same definition)
    pure_o = Ho[[r.name in ("xxx", "yyy", "zzz") for r in lat.rows]]
    pure_h = Hm[-lat.d:]
    assert np.allclose(pure_o, pure_h, atol=1e-12)


def test_d2q17_case_needs_vanishing_dropped_weights():
    card = W.Q17_CASES[0]
    with pytest.raises(H.MrtlbError) as e:
        H.Lattice(card.kind, card.c, card.cs2 * 1.01, card.free)
    assert e.value.status == H.MRTLB_EINVAL


def test_lattice_errors():
    with pytest.raises(H.MrtlbError) as e:
        H.Lattice(7, (1, 1), 0.5)
    assert e.value.status == H.MRTLB_EINVAL
    with pytest.raises(H.MrtlbError) as e:
        H.Lattice("rD2Q25", (1.5, 1.0), 1.5, (0.0, 0.0, 0.0))
    assert e.value.status == H.MRTLB_EINVAL
    with pytest.raises(H.MrtlbError) as e:      # infeasible: w1 < 0
        H.Lattice("rD2Q25", (1.5, 1.0), 1.5, (1e-3, 1e-3, 2e-2, 1e-3))
    assert e.value.status == H.MRTLB_ENUMERIC
    with pytest.raises(H.MrtlbError) as e:
        H.Lattice("rD2Q13", (1.0, -1.0), 0.5)
    assert e.value.status == H.MRTLB_EINVAL


def test_footprint():
    lat = H.Lattice(W.Q25_RECT.kind, W.Q25_RECT.c, W.Q25_RECT.cs2, W.Q25_RECT.free)
    b32 = H.footprint(lat, (4096, 4096), "fp32", "NSE_INC")
    b16 = H.footprint(lat, (4096, 4096), "fp16_dev", "NSE_INC")
    assert b32 >= 2 * 25 * 4 * 4096 * 4096
    assert b16 < 0.51 * b32
    # the gradient form of M2G keeps two slots of rho, rho u (compressible)
    # or rho_bar (incompressible) per node
    n = 64 * 64
    bf = H.footprint(lat, (64, 64), "fp32", "NSE_COMP", has_force=True)
    assert H.footprint(lat, (64, 64), "fp32", "NSE_COMP", has_force=True, m2g_form=1) - bf == 2 * 3 * n * 4
    assert H.footprint(lat, (64, 64), "fp64", "NSE_INC", m2g_form=1) - H.footprint(lat, (64, 64), "fp64", "NSE_INC") \
        == 2 * n * 8
    # a forced solve reserves d + 1 node fields: the force and a mass-source field
    assert bf - H.footprint(lat, (64, 64), "fp32", "NSE_COMP") == 3 * n * 4


def _header_struct_fields(name):
    """(field, C type, array length) of the typedef'd struct ``name`` in
    include/mrtlb.h, in declaration order (comments stripped)."""
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "include", "mrtlb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    m = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    fields = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        decl = decl.replace("const ", "")
        ctype, names = decl.split(None, 1)     # "int* e" -> ("int*", "e")
        for item in names.split(","):
            item = item.strip()
            if item.startswith("*"):
                fields.append((item[1:], ctype + "*", 1))
                continue
            arr = re.match(r"(\w+)\[(\d+)\]", item)
            fields.append((arr.group(1), ctype, int(arr.group(2))) if arr else (item, ctype, 1))
    return fields


@pytest.mark.parametrize("name", ["mrtlb_lattice_desc", "mrtlb_model_desc"])
def test_binding_structs_match_the_header(name):
    """The ctypes mirrors of the descriptor structs have the header's
    fields, types and order, so the library reads what the binding writes."""
    cls = getattr(H, name)
    ctype_of = {"int": ctypes.c_int, "double": ctypes.c_double, "int*": ctypes.POINTER(ctypes.c_int),
                "double*": ctypes.POINTER(ctypes.c_double)}
    want = _header_struct_fields(name)
    got = cls._fields_
    assert [f for f, _, _ in want] == [f for f, _ in got]
    for (f, ct, n), (_, t) in zip(want, got):
        assert t == (ctype_of[ct] * n if n > 1 else ctype_of[ct]), f


def test_population_bytes_follow_the_documented_layout():
    """ny*nz grid rows of b population rows, each nx rounded up to 32 elements."""
    q25 = H.Lattice(W.Q25_RECT.kind, W.Q25_RECT.c, W.Q25_RECT.cs2, W.Q25_RECT.free)
    assert H.population_bytes(q25, (70, 50), "fp32") == 25 * 70 * 64 * 4
    assert H.population_bytes(q25, (7, 300), "i16_dev") == 25 * 7 * 320 * 2
    q53 = H.Lattice(W.Q53_RECT.kind, W.Q53_RECT.c, W.Q53_RECT.cs2, W.Q53_RECT.free)
    assert H.population_bytes(q53, (6, 10, 70), "fp64") == 53 * 60 * 96 * 8


def _shuffled(card, seed=0):
    lat = OL.make_lattice(card.kind, card.c, card.cs2, card.free)
    perm = np.random.default_rng(seed).permutation(lat.b)
    return lat.e[perm], lat.w[perm]


@pytest.mark.parametrize("card", [W.Q25_RECT, W.Q33_CUBIC, W.Q21K_RECT], ids=lambda c: c.kind)
def test_custom_lattice_matches_oracle(card):
    """A user-supplied velocity set (a known lattice in shuffled order):
    the library keeps e and w and builds W-orthogonal rows spanning the
    oracle's, with the same corrected pure rows."""
    e, w = _shuffled(card, 5)
    q = H.Lattice("custom", card.c, card.cs2, e=e, w=w).query()
    lat = OL.custom_lattice("custom", card.c, card.cs2, e, w)
    assert np.array_equal(q["e"], e) and np.array_equal(q["w"], w)
    Hm = q["H"]
    G = (Hm * w) @ Hm.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-12 * np.abs(np.diag(G)).max()
    pure_o = lat.H()[[r.name in ("xxx", "yyy", "zzz") for r in lat.rows]]
    assert np.allclose(pure_o, Hm[-lat.d:], atol=1e-12)


def test_custom_lattice_errors():
    e, w = _shuffled(W.Q25_RECT)
    for kw, status in [(dict(e=e, w=w * 1.01), H.MRTLB_EINVAL),                  # weights do not sum to 1
                       (dict(e=e * 3, w=w), H.MRTLB_EINVAL),                      # |e| > 8
                       (dict(e=e[:, :1].repeat(2, 1), w=w), H.MRTLB_ENUMERIC)]:   # rows not orthogonal
        with pytest.raises(H.MrtlbError) as err:
            H.Lattice("custom", W.Q25_RECT.c, W.Q25_RECT.cs2, **kw)
        assert err.value.status == status
    # the single-layer D2Q9 has no independent pure third-order rows
    q9 = OL.make_lattice("D2Q9", (1.0, 1.0), 1 / 3)
    with pytest.raises(H.MrtlbError) as err:
        H.Lattice("custom", (1.0, 1.0), 1 / 3, e=q9.e, w=q9.w)
    assert err.value.status == H.MRTLB_ENUMERIC
