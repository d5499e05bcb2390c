"""Streaming alone (mrtlb_stream_only): the pull streaming of eq. 2-2 with no
collision moves every stored number from x - e_j to x unchanged, so the
populations read back after n passes equal the oracle's periodic streaming
applied n times to the populations read before, exactly, for every storage
(the read-out decodes a stored number the same way wherever it sits).

The cases cover the step kernel's launch shapes: one node per lane with row
pitches that keep a wavefront in one grid row (the wave-uniform gather) and
pitches that do not, 2 and 4 nodes per lane on long 2D rows, the periodic
x-edges, both tile orders, and the full-size rD3Q53 grid of the benchmark.
"""

import numpy as np
import pytest

from oracle import lattice as OL
from oracle import model as OM
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


def _fields(card, shape, seed):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.02 * rng.normal(size=shape)
    u = 0.03 * rng.normal(size=(card.d,) + tuple(shape))
    return rho, u


def _check(ctx, card, shape, storage, eq="NSE_COMP", passes=3, seed=3):
    lat = OL.make_lattice(card.kind, card.c, card.cs2, card.free)
    kw = dict(D0=0.1) if eq == "NCDE" else dict(m30=card.kind not in ("D2Q9", "D3Q27"))
    s = H.Solve(ctx, hip_lattice(card), hip_model(eq, RATES, **kw), shape, storage)
    rho, u = _fields(card, shape, seed)
    s.init_fields(rho if eq != "NCDE" else rho - 1.0, None if eq == "NCDE" else u)
    before = s.read_populations()
    steps0 = s.steps
    s.stream_only(passes)
    after = s.read_populations()
    assert s.steps == steps0                       # not a step of the method
    want = before
    for _ in range(passes):
        want = OM.stream(lat, want)
    s.close()
    assert np.array_equal(after, want)


@pytest.mark.parametrize("card,shape", [
    (W.Q25_RECT, (12, 70)),        # pitch 96: wavefronts cross rows
    (W.Q25_RECT, (9, 64)),         # pitch 64: one row per wavefront
    (W.Q25_RECT, (5, 512)),        # 2 (FP32/FP64) or 4 (16-bit) nodes per lane, wave-uniform rows
    (W.Q25_RECT, (4, 600)),        # several nodes per lane, pitch 608
    (W.Q53_RECT, (6, 10, 40)),     # pitch 64
    (W.Q53_RECT, (5, 7, 33)),      # pitch 64, ragged x
    (W.Q27_RECT, (7, 5, 70)),
    (W.Q9_RECT, (37, 66)),
], ids=lambda v: v.kind if hasattr(v, "kind") else "x".join(map(str, v)))
@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp32_dev", "fp16_dev", "i16_dev", "fp32_dev_f64"])
def test_stream_only_equals_oracle_streaming(ctx, card, shape, storage):
    print("case: stream only %s %s %s" % (card.kind, shape, storage), flush=True)
    _check(ctx, card, shape, storage)


@pytest.mark.parametrize("order", ["0", "1"])
def test_stream_only_both_tile_orders(ctx, monkeypatch, order):
    """The tile order is a launch choice only (MRTLB_XCD_ORDER is read when a
    solve is created)."""
    monkeypatch.setenv("MRTLB_XCD_ORDER", order)
    print("case: stream only tile order %s" % order, flush=True)
    _check(ctx, W.Q53_RECT, (6, 10, 40), "i16_dev")
    _check(ctx, W.Q25_RECT, (4, 1024), "fp32")


def test_stream_only_ncde(ctx):
    print("case: stream only rD2Q13 NCDE", flush=True)
    _check(ctx, W.Q13_SQUARE, (37, 66), "fp32", eq="NCDE")


def test_stream_only_full_size_rd3q53(ctx):
    """The benchmark grid, rD3Q53 256^3 int16: sampled nodes after two passes
    against the populations two lattice steps upstream (periodic)."""
    card, n = W.Q53_RECT, 256
    shape = (n, n, n)
    lat = OL.make_lattice(card.kind, card.c, card.cs2, card.free)
    s = H.Solve(ctx, hip_lattice(card), hip_model("NSE_COMP", RATES), shape, "i16_dev")
    rho, u = _fields(card, shape, 5)
    print("case: stream only rD3Q53 256^3 i16_dev", flush=True)
    s.init_fields(rho, u)
    del rho, u
    before = s.read_populations()
    s.stream_only(2)
    after = s.read_populations()
    s.close()
    rng = np.random.default_rng(9)
    pts = rng.integers(0, n, size=(2000, 3))
    pts[:8] = [[0, 0, 0], [n - 1, n - 1, n - 1], [0, 1, n - 1], [1, 0, n - 2], [n - 1, 0, 0], [0, n - 1, 1],
               [n - 2, n - 1, 0], [0, 0, 1]]
    e = lat.e.astype(int)
    for z, y, x in pts:
        src = [before[j, (z - 2 * e[j, 2]) % n, (y - 2 * e[j, 1]) % n, (x - 2 * e[j, 0]) % n] for j in range(lat.b)]
        assert np.array_equal(after[:, z, y, x], np.array(src))


def test_stream_only_errors(ctx):
    card = W.Q25_RECT
    s = H.Solve(ctx, hip_lattice(card), hip_model("NSE_COMP", RATES), (8, 64), "fp32")
    with pytest.raises(H.MrtlbError) as e:
        s.stream_only(-1)
    assert e.value.status == H.MRTLB_EINVAL
    assert s.stream_only(0, timed=True) >= 0.0
    s.close()
