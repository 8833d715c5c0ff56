"""Serving loop: continuous batching of tissue simulations on one GPU.

Requests (a tissue problem plus its number of splitting steps) arrive over
time.  The server keeps every admitted tissue resident in HBM and, tick by
tick, advances all of them together by a quantum of steps in one batch
(`tissue_batch_step`: every chi/S launch covers the work items of all active
tissues).  A request is admitted as soon as a slot is free and its device
bytes (`tissue_required_bytes`) fit the memory budget; it leaves as soon as
its last step is done, its counts are read back and its buffer is released.
So requests that arrive while others run join the next tick and their work
overlaps on the device with everyone else's.

Each tissue carries its own step counter and random stream (seed, sim_id,
step index), so its result does not depend on which other tissues shared its
launches: a request gives the same bits alone and in the mix.

The loop is written against a small backend interface (`GpuBackend` below);
the tests drive the same loop with a CPU backend to check admission and
accounting.
"""
from __future__ import annotations

import collections
import heapq
import time
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    problem: dict
    n_steps: int
    arrival: float                 # seconds since the start of the run
    admitted: float | None = None
    finished: float | None = None
    steps_done: int = 0
    handle: object = None
    bytes: int = 0
    result: object = None
    events: int = 0


@dataclass
class ServeStats:
    completed: int = 0
    events: int = 0
    wall_s: float = 0.0
    max_active: int = 0
    mean_active: float = 0.0
    max_bytes: int = 0
    ticks: int = 0
    latencies: list = field(default_factory=list)
    queue_waits: list = field(default_factory=list)

    def summary(self) -> dict:
        lat = sorted(self.latencies)

        def pct(q):
            if not lat:
                return None
            k = (len(lat) - 1) * q / 100.0
            lo, hi = int(k), min(int(k) + 1, len(lat) - 1)
            return lat[lo] + (lat[hi] - lat[lo]) * (k - lo)
        return {
            "completed": self.completed, "wall_s": self.wall_s,
            "req_per_s": self.completed / self.wall_s if self.wall_s else None,
            "events_per_s": self.events / self.wall_s if self.wall_s else None,
            "latency_ms_p50": None if not lat else pct(50) * 1e3,
            "latency_ms_p99": None if not lat else pct(99) * 1e3,
            "latency_ms_mean": None if not lat else 1e3 * sum(lat) / len(lat),
            "max_active": self.max_active, "mean_active": self.mean_active,
            "max_hbm_bytes": self.max_bytes, "ticks": self.ticks,
        }


class Server:
    """Continuous-batching loop.

    backend: object with required_bytes(problem), create(problem),
      step(handles, dt, n) (advance all handles by n steps, async allowed),
      sync(), events(handle), read(handle), free(handle).
    max_bytes: HBM budget for resident tissues; max_active: slot count;
    quantum: steps per tick.
    """

    def __init__(self, backend, max_bytes: int, max_active: int = 4096, quantum: int = 10,
                 clock=time.perf_counter, keep_results: bool = False):
        self.backend = backend
        self.max_bytes = int(max_bytes)
        self.max_active = int(max_active)
        self.quantum = int(quantum)
        self.clock = clock
        self.keep_results = keep_results

    def run(self, requests, real_time: bool = True) -> tuple[ServeStats, list]:
        """Serve `requests` (sorted by arrival).  With real_time, arrivals are
        replayed against the wall clock (a request cannot be admitted before
        its arrival time); otherwise the clock is virtual and every tick
        advances it by the tick's measured duration."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: list = []  # arrived, not admitted: (arrival, rid, req)
        active: list[Request] = []
        done: list[Request] = []
        st = ServeStats()
        used = 0
        t0 = self.clock()
        vt = 0.0
        active_sum = 0
        while pending or waiting or active:
            now = (self.clock() - t0) if real_time else vt
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                heapq.heappush(waiting, (r.arrival, r.rid, r))
            # admission: oldest first, by free slots and free HBM
            while waiting and len(active) < self.max_active:
                r = waiting[0][2]
                need = self.backend.required_bytes(r.problem)
                if need > self.max_bytes:
                    raise ValueError(f"request {r.rid} needs {need} B, over the whole budget")
                if used + need > self.max_bytes:
                    break
                heapq.heappop(waiting)
                r.bytes = need
                r.handle = self.backend.create(r.problem)
                r.admitted = now
                used += need
                active.append(r)
            if not active:
                # idle: jump to the next arrival
                if not pending:
                    break
                if real_time:
                    delay = pending[0].arrival - (self.clock() - t0)
                    if delay > 0:
                        time.sleep(min(delay, 0.05))
                else:
                    vt = max(vt, pending[0].arrival)
                continue
            st.max_active = max(st.max_active, len(active))
            st.max_bytes = max(st.max_bytes, used)
            active_sum += len(active)
            # one tick: every active tissue advances by up to one quantum;
            # tissues needing fewer steps than the quantum finish this tick
            tick_start = self.clock()
            q = min([self.quantum] + [r.n_steps - r.steps_done for r in active])
            dt = active[0].problem["dt"]
            same_dt = all(r.problem["dt"] == dt for r in active)
            if same_dt:
                self.backend.step([r.handle for r in active], dt, q)
            else:
                by_dt = collections.defaultdict(list)
                for r in active:
                    by_dt[r.problem["dt"]].append(r.handle)
                for d, hs in by_dt.items():
                    self.backend.step(hs, d, q)
            self.backend.sync()
            st.ticks += 1
            finished_now = self.clock()
            if not real_time:
                vt += finished_now - tick_start
            end = (finished_now - t0) if real_time else vt
            still = []
            for r in active:
                r.steps_done += q
                if r.steps_done >= r.n_steps:
                    r.events = self.backend.events(r.handle)
                    if self.keep_results:
                        r.result = self.backend.read(r.handle)
                    self.backend.free(r.handle)
                    r.handle = None
                    used -= r.bytes
                    r.finished = end
                    st.completed += 1
                    st.events += r.events
                    st.latencies.append(r.finished - r.arrival)
                    st.queue_waits.append(r.admitted - r.arrival)
                    done.append(r)
                else:
                    still.append(r)
            active = still
        st.wall_s = (self.clock() - t0) if real_time else vt
        st.mean_active = active_sum / st.ticks if st.ticks else 0.0
        return st, done


class GpuBackend:
    """The C-ABI library as a serving backend: one Tissue per request (its
    own device buffer) and one Batch per distinct active set, rebuilt only
    when the set changes."""

    def __init__(self, device="cuda:0", stream=None, graph_chunk: int = 0):
        import torch

        from . import tissue as T
        self.T = T
        self.torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.graph_chunk = graph_chunk
        self._batch = None
        self._batch_key = None

    def required_bytes(self, problem):
        return self.T.required_bytes(problem) + 256

    def create(self, problem):
        t = self.T.Tissue(problem, device=self.device, stream=self.stream)
        return t

    def step(self, handles, dt, n):
        key = tuple(id(h) for h in handles)
        if key != self._batch_key:
            if self._batch is not None:
                self._batch.close()
            self._batch = self.T.Batch(handles, device=self.device, stream=self.stream)
            self._batch_key = key
        self._batch.step(dt, n)

    def sync(self):
        if self._batch is not None:
            self._batch.sync()

    def events(self, h):
        st = h.stats()
        return st["chi_events"] + st["s_events"]

    def read(self, h):
        return h.read_counts()

    def free(self, h):
        if self._batch is not None:
            self._batch.close()
            self._batch, self._batch_key = None, None
        h.close()
        h.buffer = None


def requests_from_workload(n: int, seed: int = 5, rate_hz: float = 200.0, n_steps: int = 100,
                           first: int = 0) -> list[Request]:
    """The serving workload: Poisson arrivals, request q = config5_request(q)."""
    from . import workloads as W
    arr = W.config5_arrivals(seed=seed, n_requests=first + n, rate_hz=rate_hz)
    out = []
    for q in range(first, first + n):
        p = W.config5_request(q, seed=seed, n_steps=n_steps)
        out.append(Request(rid=q, problem=p, n_steps=n_steps, arrival=float(arr[q] - arr[first])))
    return out
