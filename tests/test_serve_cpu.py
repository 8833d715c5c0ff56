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
    """A request that can never fit the budget is ended as rejected and the
    loop goes on serving the others."""
    reqs = _requests(4)
    be = OracleBackend(oracle_lib)
    sizes = [be.required_bytes(r.problem) for r in reqs]
    big = int(np.argmax(sizes))
    budget = sorted(sizes)[-2]  # everything but the largest fits
    srv = serve.Server(be, max_bytes=budget, quantum=2)
    st, done = srv.run(reqs, real_time=False)
    by = {r.rid: r for r in done}
    assert by[reqs[big].rid].status == "rejected" and "budget" in by[reqs[big].rid].error
    assert st.rejected == 1 and st.completed == len(reqs) - 1 and be.live == {}
    assert all(r.status == "done" for r in done if r.rid != reqs[big].rid)


def test_budget_from_free_memory_binds(oracle_lib):
    """Without an explicit budget the server takes the backend's free memory
    minus a margin; a budget of twice the largest request binds (requests
    wait for others to leave) and holds, and every request still completes
    with its own result."""
    reqs = _requests(8)
    be = OracleBackend(oracle_lib)
    two = max(be.required_bytes(r.problem) for r in reqs) * 2
    be.free_bytes = lambda: two + 1000
    srv = serve.Server(be, margin_bytes=1000, quantum=3, keep_results=True)
    assert srv.max_bytes == two
    st, done = srv.run(reqs, real_time=False)
    assert st.completed == 8 and st.max_bytes <= two and be.live == {}
    assert max(st.queue_waits) > 0
    for r in done:
        assert np.array_equal(r.result, oracle_lib.run(r.problem, r.problem["dt"], r.n_steps).counts)


def test_ebusy_when_the_waiting_queue_is_full(oracle_lib):
    """submit answers EBUSY while the waiting queue is full (a request that
    cannot be admitted now: the budget holds one at a time); the replay
    tries again later, and every request completes.  Ticks take 50 ms on a
    fake clock and requests arrive 10 ms apart, so the queue fills."""
    clock = FakeClock()
    reqs = _requests(6)
    be = TickBackend(oracle_lib, clock, 0.05)
    one = max(be.required_bytes(r.problem) for r in reqs)
    srv = serve.Server(be, max_bytes=one, quantum=2, max_waiting=1, clock=clock, sleep=clock.sleep)
    assert srv.submit(reqs[0]) == serve.OK
    assert srv.submit(reqs[1]) == serve.EBUSY
    st, done = srv.run(reqs, real_time=True)
    assert st.completed == 6 and st.busy_retries > 0 and be.live == {}
    assert sorted(r.rid for r in done) == list(range(6))


class SlowBackend(OracleBackend):
    """Ticks take time on a fake clock: a tick containing request 2 takes
    1 s, any other 10 ms."""

    def __init__(self, oracle_lib, clock):
        super().__init__(oracle_lib)
        self.clock = clock
        self.until = 0.0
        self.rid_of = {}

    def create(self, p, lane):
        h = super().create(p, lane)
        self.rid_of[id(h)] = p["sim_id"]
        return h

    def step(self, lane, handles, dt, n, finishing=()):
        super().step(lane, handles, dt, n, finishing)
        slow = any(self.rid_of[id(h)] == 2 for h in handles)
        self.until = self.clock.t + (1.0 if slow else 0.01)

    def busy(self, lane):
        return self.clock.t < self.until


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4
        return self.t

    def sleep(self, s):
        self.t += s


class TickBackend(OracleBackend):
    """Every tick takes tick_s on a fake clock."""

    def __init__(self, oracle_lib, clock, tick_s):
        super().__init__(oracle_lib)
        self.clock = clock
        self.tick_s = tick_s
        self.until = 0.0

    def step(self, lane, handles, dt, n, finishing=()):
        super().step(lane, handles, dt, n, finishing)
        self.until = self.clock.t + self.tick_s

    def busy(self, lane):
        return self.clock.t < self.until


def test_tick_deadline_fails_the_requests_and_goes_on(oracle_lib):
    """A tick over its deadline marks the requests in it failed (released
    when the tick ends, never retried); requests in later ticks complete."""
    clock = FakeClock()
    reqs = [serve.Request(rid=q, problem=dict(W.config5_request(q, side_hi=6.0, n_steps=4), sim_id=q),
                          n_steps=4, arrival=0.05 * q) for q in range(5)]
    be = SlowBackend(oracle_lib, clock)
    srv = serve.Server(be, max_bytes=10 ** 12, quantum=4, max_active=1, clock=clock,
                       sleep=clock.sleep, tick_deadline_s=0.5, keep_results=True)
    st, done = srv.run(reqs, real_time=True)
    by = {r.rid: r for r in done}
    assert by[2].status == "failed" and "deadline" in by[2].error
    assert st.failed == 1 and st.completed == 4 and be.live == {}
    for q in (0, 1, 3, 4):
        r = by[q]
        assert r.status == "done"
        assert np.array_equal(r.result, oracle_lib.run(r.problem, r.problem["dt"], r.n_steps).counts)


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


def test_cancellation_waiting_and_active(oracle_lib):
    """A cancelled request ends as cancelled and is released -- a waiting
    one at once, an active one when its lane's tick ends, one not yet
    arrived when it arrives; the others complete with their own results."""
    clock = FakeClock()
    reqs = [serve.Request(rid=q, problem=dict(W.config5_request(q, side_hi=6.0, n_steps=4), sim_id=q),
                          n_steps=4, arrival=0.05 * q) for q in range(6)]
    be = SlowBackend(oracle_lib, clock)
    srv = serve.Server(be, max_bytes=10 ** 12, quantum=4, max_active=1, clock=clock,
                       sleep=clock.sleep, keep_results=True)
    # at 0.3 s request 2 is in its (1 s) tick and 3, 4 are waiting; 5 arrives later
    st, done = srv.run(reqs, real_time=True, cancels=[(0.3, 2), (0.3, 4), (0.3, 5)])
    by = {r.rid: r for r in done}
    assert by[2].status == "cancelled" and by[2].admitted is not None and by[2].finished >= 1.0
    assert by[4].status == "cancelled" and by[4].admitted is None
    assert by[5].status == "cancelled" and by[5].admitted is None
    assert st.cancelled == 3 and st.completed == 3 and be.live == {}
    for q in (0, 1, 3):
        r = by[q]
        assert r.status == "done"
        assert np.array_equal(r.result, oracle_lib.run(r.problem, r.problem["dt"], r.n_steps).counts)

