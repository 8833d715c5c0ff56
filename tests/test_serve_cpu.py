"""Serving loop logic on the CPU: admission by free slots and memory,
oldest-first order, every request completes with its own result, accounting
of latency and concurrency.  The backend here runs the CPU oracle (test
infrastructure); the GPU test drives the same loop through the C-ABI."""
import numpy as np

from paper_1806_10889_amd import serve
from paper_1806_10889_amd import workloads as W


class OracleBackend:
    """Runs every tick at once (never busy); `lanes` lanes share it."""

    def __init__(self, oracle_lib, bytes_per_voxel=100, lanes=1):
        self.o = oracle_lib
        self.lanes = lanes
        self.bpv = bytes_per_voxel
        self.live = {}
        self.created = []
        self.used_peak = 0

    def required_bytes(self, p):
        return W.n_voxels(p) * self.bpv

    def create(self, p, lane):
        h = object()
        self.live[id(h)] = dict(p=p, counts=p["init_counts"].copy(), step=p["start_step"], ev=0, h=h)
        self.created.append(p["sim_id"])
        return h

    def step(self, lane, handles, dt, n, finishing=()):
        for h in handles:
            s = self.live[id(h)]
            r = self.o.run(s["p"], dt, n, counts=s["counts"], start_step=s["step"])
            s["counts"], s["step"], s["ev"] = r.counts, s["step"] + n, s["ev"] + r.chi_events + r.s_events

    def busy(self, lane):
        return False

    def sync(self, lane):
        pass

    def events(self, h):
        return self.live[id(h)]["ev"]

    def read(self, h):
        return self.live[id(h)]["counts"].copy()

    def free(self, lane, h):
        del self.live[id(h)]


def _requests(n, steps=6):
    reqs = []
    for q in range(n):
        p = W.config5_request(q, side_hi=6.0, n_steps=steps)
        reqs.append(serve.Request(rid=q, problem=p, n_steps=steps + (q % 3), arrival=0.01 * q))
    return reqs


def test_admission_budget_and_results(oracle_lib):
    reqs = _requests(12)
    be = OracleBackend(oracle_lib)
    budget = max(be.required_bytes(r.problem) for r in reqs) * 3
    srv = serve.Server(be, max_bytes=budget, max_active=4, quantum=4, keep_results=True)
    st, done = srv.run(reqs, real_time=False)
    assert st.completed == len(reqs) and len(done) == len(reqs)
    assert st.max_active <= 4 and st.max_bytes <= budget
    assert be.live == {}
    # oldest first: admission order follows arrival order
    assert be.created == sorted(be.created)
    for r in done:
        alone = oracle_lib.run(r.problem, r.problem["dt"], r.n_steps)
        assert np.array_equal(r.result, alone.counts), r.rid
        assert r.events == alone.chi_events + alone.s_events
        assert r.finished >= r.admitted >= r.arrival
    s = st.summary()
    assert s["latency_ms_p99"] >= s["latency_ms_p50"] > 0


def test_oversized_request_is_rejected(oracle_lib):
    reqs = _requests(2)
    be = OracleBackend(oracle_lib)
    srv = serve.Server(be, max_bytes=1, quantum=2)
    try:
        srv.run(reqs, real_time=False)
    except ValueError as e:
        assert "budget" in str(e)
    else:
        raise AssertionError("expected rejection")


def test_lanes_route_by_chain_estimate_and_keep_results(oracle_lib):
    """Several lanes: every request completes with its own result, heavier
    requests (by the estimate of their busiest cell's events per step) go to
    higher lanes, and the slot and byte limits hold over all lanes."""
    reqs = _requests(16)
    be = OracleBackend(oracle_lib, lanes=3)
    budget = max(be.required_bytes(r.problem) for r in reqs) * 5
    srv = serve.Server(be, max_bytes=budget, max_active=6, quantum=3, keep_results=True)
    st, done = srv.run(reqs, real_time=False)
    assert st.completed == len(reqs) and st.lanes == 3
    assert st.max_active <= 6 and st.max_bytes <= budget and be.live == {}
    for r in done:
        alone = oracle_lib.run(r.problem, r.problem["dt"], r.n_steps)
        assert np.array_equal(r.result, alone.counts), r.rid
    # routing is monotone in the estimate among requests seen in order
    est = {r.rid: serve.chain_estimate(r.problem) for r in done}
    lanes = {r.rid: r.lane for r in done}
    assert len(set(lanes.values())) > 1
    seen = []
    for rid in sorted(est):  # arrival order
        below = sum(1 for e in seen if e < est[rid])
        assert lanes[rid] == min(2, int(below / max(len(seen), 1) * 3))
        seen.append(est[rid])


def test_chain_estimate_grows_with_rates_and_mesh():
    p = W.config5_request(3, side_hi=6.0, n_steps=2)
    q = dict(p)
    q["rates"] = p["rates"] * 10.0
    assert serve.chain_estimate(q) > serve.chain_estimate(p)
    big = dict(p)
    big["mesh_w"] = np.full_like(p["mesh_w"], 4)
    big["mesh_h"] = np.full_like(p["mesh_h"], 4)
    assert serve.chain_estimate(big) >= serve.chain_estimate(p)
