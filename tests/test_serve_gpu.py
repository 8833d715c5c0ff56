"""Serving on the GPU: continuous batching through the C-ABI.  Each served
result is bit-identical to the same request run alone, and to the oracle."""
import numpy as np
import pytest

from paper_1806_10889_amd import serve
from paper_1806_10889_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone_and_oracle(oracle_lib):
    from paper_1806_10889_amd import tissue as T
    reqs = []
    for q in range(40):
        steps = 12 + (q % 5)
        p = W.config5_request(q, side_hi=20.0, n_steps=steps)
        reqs.append(serve.Request(rid=q, problem=p, n_steps=steps, arrival=0.002 * q))
    be = serve.GpuBackend(lanes=2)  # two lanes fit the default four hardware queues
    budget = sum(be.required_bytes(r.problem) for r in reqs) // 4
    srv = serve.Server(be, max_bytes=budget, max_active=12, quantum=5, keep_results=True)
    st, done = srv.run(reqs, real_time=False)
    assert st.completed == 40 and st.max_active > 1 and st.max_bytes <= budget
    by_id = {r.rid: r for r in done}
    for q in [0, 3, 7, 12, 19, 26, 33, 39]:
        r = by_id[q]
        t = T.Tissue(r.problem)
        t.step(r.problem["dt"], r.n_steps)
        assert np.array_equal(r.result, t.read_counts()), q
        st1 = t.stats()
        assert r.events == st1["chi_events"] + st1["s_events"]
        t.close()
    for q in [0, 19, 39]:
        r = by_id[q]
        o = oracle_lib.run(r.problem, r.problem["dt"], r.n_steps)
        assert np.array_equal(r.result, o.counts), q
