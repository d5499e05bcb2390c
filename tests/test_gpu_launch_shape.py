"""The step kernel's launch shape as the library chooses it
(mrtlb_solve_launch_shape): nodes per lane, tile order over the XCDs and the
occupancy cap, on the MI355X (256 compute units).  These are measured
heuristics; the cases pin the choices at the grids they were measured on, so
that a change to them shows here.  Results do not depend on the launch shape
(test_gpu_parity checks that bit for bit); only speed does.  No solve is
stepped: creation alone fixes the shape.
"""

import pytest

from paper_2512_16230_amd import _mrtlb as H
from paper_2512_16230_amd import workloads as W

from helpers import hip_lattice, hip_model

pytestmark = pytest.mark.gpu

RATES = W.Rates(1.6, 1.3, 1.25, 1.1, 1.15, 1.2)


@pytest.fixture(scope="module")
def ctx():
    c = H.Context(0)
    yield c
    c.close()


def _shape(ctx, card, shape, storage, eq="NSE_COMP", custom=False, **kw):
    lat = hip_lattice(card)
    if custom:
        q = lat.query()
        lat = H.Lattice("custom", card.c, card.cs2, e=q["e"], w=q["w"])
    if eq == "NSE_COMP":
        kw.setdefault("m30", card.kind not in ("D2Q9", "D3Q27"))
    s = H.Solve(ctx, lat, hip_model(eq, RATES, **kw), shape, storage)
    out = s.launch_shape()
    s.close()
    return out


CASES = [
    # 2D NSE, 32/64-bit storage: two nodes per lane, XCD ranges, two (b >= 25) or three workgroups per CU
    ((W.Q25_RECT, (4096, 4096), "fp32_dev", {}), (2, "xcd", 2, 32768)),
    ((W.Q25_RECT, (4096, 4096), "fp32", {}), (2, "xcd", 2, 32768)),
    ((W.Q9_RECT, (4096, 4096), "fp32", {}), (2, "xcd", 3, 32768)),
    ((W.Q25_RECT, (2048, 2048), "fp32_dev", {}), (2, "xcd", 2, 8192)),
    # below eight rounds of the capped residency: no cap
    ((W.Q25_RECT, (1024, 1024), "fp32_dev", {}), (2, "xcd", 0, 2048)),
    ((W.Q9_RECT, (1024, 1024), "fp32", {}), (2, "xcd", 0, 2048)),
    # the gradient form: one node per lane, three per CU
    ((W.Q25_RECT, (4096, 4096), "fp32_dev", dict(m2g_form=1)), (1, "xcd", 3, 65536)),
    # 2D 16-bit: four nodes per lane, dispatch order, no cap
    ((W.Q25_RECT, (4096, 4096), "i16_dev", {}), (4, "dispatch", 0, 16384)),
    ((W.Q9_RECT, (4096, 4096), "fp16_dev", {}), (4, "dispatch", 0, 16384)),
    # 3D: one node per lane, dispatch order; two per CU at >= 180 stored bytes per node, else three
    ((W.Q53_RECT, (256, 256, 256), "fp32", {}), (1, "dispatch", 2, 65536)),
    ((W.Q53_RECT, (128, 128, 128), "fp32", {}), (1, "dispatch", 2, 8192)),
    ((W.Q53_RECT, (96, 96, 96), "fp32", {}), (1, "dispatch", 0, 3456)),
    ((W.Q53_RECT, (64, 64, 64), "fp32", {}), (1, "dispatch", 0, 1024)),
    ((W.Q53_RECT, (256, 256, 256), "fp32", dict(m2g_form=1)), (1, "dispatch", 3, 65536)),
    ((W.Q53_RECT, (256, 256, 256), "i16_dev", {}), (1, "dispatch", 0, 65536)),
    ((W.Q27_RECT, (256, 256, 256), "fp32", {}), (1, "dispatch", 3, 65536)),
    ((W.Q27_RECT, (256, 256, 256), "fp64", {}), (1, "dispatch", 2, 65536)),
    ((W.Q33_CUBIC, (128, 128, 128), "fp32", {}), (1, "dispatch", 3, 8192)),
]


@pytest.mark.parametrize("case,want", CASES,
                         ids=["%s-%s-%s%s" % (c[0].kind, "x".join(map(str, c[1])), c[2], "-m2g" if c[3] else "")
                              for c, _ in CASES])
def test_nse_launch_shape(ctx, case, want):
    card, shape, storage, kw = case
    got = _shape(ctx, card, shape, storage, **kw)
    print("case: launch shape %s %s %s %s -> %s" % (card.kind, shape, storage, kw, got), flush=True)
    assert (got["nodes_per_lane"], got["tile_order"], got["wg_per_cu"], got["workgroups"]) == want


def test_ncde_cde_launch_shape(ctx):
    card = W.Q13_SQUARE
    # 2D NCDE/CDE: one node per lane, four per CU with 32/64-bit storage on large grids
    got = _shape(ctx, card, (4096, 4096), "fp32", eq="CDE")
    assert (got["nodes_per_lane"], got["tile_order"], got["wg_per_cu"]) == (1, "xcd", 4)
    got = _shape(ctx, card, (4096, 4096), "i16_dev", eq="CDE")
    assert (got["nodes_per_lane"], got["tile_order"], got["wg_per_cu"]) == (1, "dispatch", 0)
    got = _shape(ctx, card, (1024, 1024), "fp32", eq="NCDE", D0=0.1)
    assert (got["wg_per_cu"], got["workgroups"]) == (0, 4096)
    got = _shape(ctx, card, (2048, 2048), "fp32", eq="NCDE", D0=0.1)
    assert (got["wg_per_cu"], got["workgroups"]) == (4, 16384)
    # 3D CDE: the 3D rule
    got = _shape(ctx, W.Q53_RECT, (256, 256, 256), "fp32", eq="CDE")
    assert got["wg_per_cu"] == 2
    got = _shape(ctx, W.Q33_CUBIC, (256, 256, 256), "fp32", eq="CDE")
    assert got["wg_per_cu"] == 3


def test_user_supplied_lattice_launch_shape(ctx):
    """One node per lane and no occupancy cap."""
    got = _shape(ctx, W.Q25_RECT, (4096, 4096), "fp32_dev", custom=True)
    assert (got["nodes_per_lane"], got["wg_per_cu"]) == (1, 0)


def test_environment_overrides(ctx, monkeypatch):
    monkeypatch.setenv("MRTLB_STEP_WG_PER_CU", "3")
    monkeypatch.setenv("MRTLB_XCD_ORDER", "0")
    monkeypatch.setenv("MRTLB_STEP_VEC", "4")
    got = _shape(ctx, W.Q25_RECT, (64, 64), "fp32")
    assert (got["nodes_per_lane"], got["tile_order"], got["wg_per_cu"], got["workgroups"]) == (4, "dispatch", 3, 4)
    monkeypatch.setenv("MRTLB_STEP_WG_PER_CU", "0")
    monkeypatch.setenv("MRTLB_XCD_ORDER", "1")
    monkeypatch.delenv("MRTLB_STEP_VEC")
    got = _shape(ctx, W.Q25_RECT, (4096, 4096), "fp32")
    assert (got["nodes_per_lane"], got["tile_order"], got["wg_per_cu"]) == (2, "xcd", 0)


def test_launch_shape_errors():
    with pytest.raises(H.MrtlbError) as e:
        H._check(H.lib().mrtlb_solve_launch_shape(None, None, None, None, None))
    assert e.value.status == H.MRTLB_EINVAL
