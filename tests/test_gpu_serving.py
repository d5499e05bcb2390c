"""Served requests on the GPU: every result equals the same request run
alone (same kernels, no cross-solve arithmetic: bit for bit)."""

import numpy as np
import pytest

from paper_2512_16230_amd import serving as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["i16_dev", "bf16_dev", "fp32"])
def test_served_results_equal_solo_runs(storage):
    reqs = S.request_stream(10, rate=2000.0, seed=11, storage=storage, steps=(20, 80),
                            q25=(64, 160), q13=(128, 200), q33=(24, 40))
    print("case: serving 10 mixed requests, %s" % storage, flush=True)
    ex = S.GpuExecutor(hbm_budget=256 << 20)
    st = S.Server(ex, max_chunk=16, keep_values=True).run(reqs, real_time=True)
    assert all(r.error is None for r in st.results), [r.error for r in st.results if r.error]
    assert st.max_resident >= 2
    for q, r in zip(sorted(reqs, key=lambda q: q.rid), st.results):
        q.payload = S.make_payload(q)
        h = ex.create(q)
        ex.step([h], [q.steps])
        solo = ex.read(h, q)
        ex.release(h)
        assert np.array_equal(solo[0], r.value[0])
        if solo[1] is not None:
            assert np.array_equal(solo[1], r.value[1])
    s = st.summary()
    assert s["p99_s"] >= s["p50_s"] > 0
    ex.close()
