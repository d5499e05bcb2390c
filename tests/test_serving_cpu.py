"""Scheduling logic of the continuous-batching server, on a simulated
device (no GPU): completion, exact step counts, FIFO admission by HBM
footprint, continuous admission while others run, failure isolation and
the latency statistics."""

import numpy as np

from paper_2512_16230_amd import serving as S
from paper_2512_16230_amd import workloads as W


def _stream(n=60, rate=200.0, seed=1):
    return S.request_stream(n, rate, seed=seed)


def test_every_request_completes_with_its_step_count():
    reqs = _stream()
    ex = S.SimExecutor(hbm_budget=64 << 30)
    st = S.Server(ex, max_chunk=64, keep_values=True).run(reqs, real_time=False)
    assert len(st.results) == len(reqs)
    for r, q in zip(st.results, sorted(reqs, key=lambda q: q.rid)):
        assert r.error is None
        assert r.value[0] == q.steps           # no overshoot, no shortfall
        assert r.finished >= r.admitted >= r.arrival


def test_admission_by_footprint_and_fifo():
    reqs = _stream(80, rate=400.0, seed=2)
    budget = 2 << 30
    ex = S.SimExecutor(hbm_budget=budget)
    st = S.Server(ex).run(reqs, real_time=False)
    assert st.max_bytes <= budget
    ok = [r for r in st.results if r.error is None]
    # admission times follow arrival order (strict FIFO)
    adm = [r.admitted for r in sorted(ok, key=lambda r: r.arrival)]
    assert all(a <= b + 1e-12 for a, b in zip(adm, adm[1:]))
    # the budget binds: some requests waited for memory
    assert any(r.admitted > r.arrival + 1e-9 for r in ok)


def test_oversized_request_is_rejected_alone():
    reqs = _stream(20, seed=3)
    big = S.Request(999, reqs[5].arrival, W.Q25_RECT, "NSE_INC", (40000, 40000), 10, "bf16_dev",
                    W.rates_tau(0.8), 0)
    ex = S.SimExecutor(hbm_budget=8 << 30)
    st = S.Server(ex).run(reqs + [big], real_time=False)
    errs = [r for r in st.results if r.error]
    assert [r.rid for r in errs] == [999]
    assert sum(r.error is None for r in st.results) == len(reqs)


def test_continuous_batching_overlaps_requests():
    reqs = _stream(40, rate=300.0, seed=4)
    ex = S.SimExecutor(hbm_budget=64 << 30)
    st = S.Server(ex).run(reqs, real_time=False)
    assert st.max_resident > 3
    # some request was admitted while an earlier one was still resident
    res = sorted(st.results, key=lambda r: r.admitted)
    assert any(b.admitted < a.finished for a, b in zip(res, res[1:]))


def test_device_error_isolated_to_its_request():
    reqs = _stream(30, seed=5)
    ex = S.SimExecutor(hbm_budget=64 << 30, fail_on={7, 11})
    st = S.Server(ex, keep_values=True).run(reqs, real_time=False)
    bad = sorted(r.rid for r in st.results if r.error)
    assert bad == [7, 11]
    good = {r.rid: r for r in st.results if r.error is None}
    for q in reqs:
        if q.rid not in (7, 11):
            assert good[q.rid].value[0] == q.steps


def test_single_request_latency_is_its_work():
    q = _stream(1, seed=6)[0]
    ex = S.SimExecutor(hbm_budget=64 << 30, bandwidth=1e12)
    st = S.Server(ex, max_chunk=37).run([q], real_time=False)
    assert st.chunks == -(-q.steps // 37)
    work = 2 * S.B_OF[q.card.kind] * S.STORE_BYTES[q.storage] * q.nodes * q.steps / 1e12
    assert abs(st.results[0].latency - work) < 1e-12
    s = st.summary()
    assert abs(s["p50_s"] - work) < 1e-12


def test_summary_percentiles():
    reqs = _stream(50, seed=7)
    st = S.Server(S.SimExecutor(hbm_budget=64 << 30)).run(reqs, real_time=False)
    lat = np.array([r.latency for r in st.results])
    s = st.summary()
    assert s["p50_s"] == float(np.percentile(lat, 50))
    assert s["p99_s"] == float(np.percentile(lat, 99))
    assert s["requests"] == 50 and s["failed"] == 0


def test_payload_failure_fails_its_request_only():
    """A payload that cannot be made (the producer thread raises) fails that
    request; admission does not wait for it forever."""

    class Faulty(S.SimExecutor):
        needs_payload = True

        def prepare(self, req):
            if req.rid == 3:
                raise RuntimeError("bad payload")
            return {"rho_or_phi": None, "u": None, "force": None}

    reqs = S.request_stream(8, rate=1000.0, seed=5, steps=(20, 40), q25=(64, 96), q13=(128, 160), q33=(24, 32))
    st = S.Server(Faulty(hbm_budget=1 << 40), max_chunk=8).run(reqs, real_time=False)
    assert len(st.results) == 8
    bad = [r for r in st.results if r.error is not None]
    assert [r.rid for r in bad] == [3] and "bad payload" in bad[0].error
