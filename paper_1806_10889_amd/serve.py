"""Serving loop: continuous batching of tissue simulations on one GPU.

Requests (a tissue problem plus its number of splitting steps) arrive over
time.  The server keeps every admitted tissue resident in HBM and advances
them in batches (`tissue_batch_step`: every chi/S launch covers the work
items of all the batch's tissues) by a quantum of steps per tick.  A request
is admitted as soon as a slot is free and its device bytes
(`tissue_required_bytes`) fit the memory budget; it leaves as soon as its
last step is done, its counts are read back and its buffer is released.

The requests are spread over independent lanes, each with its own stream,
batch and tick: a tick's duration is set by the cell with the longest event
chain in the batch, so requests are routed by an estimate of that chain (the
expected events per step of their busiest cell) and light requests do not
wait on heavy ones.  While the device runs one lane's tick, the host
finishes other lanes' ticks, creates newly admitted tissues and launches the
next ticks.

Each tissue carries its own step counter and random stream (seed, sim_id,
step index), so its result does not depend on which lane or which other
tissues shared its launches: a request gives the same bits alone and in the
mix.

The loop is written against a small backend interface (`GpuBackend` below);
the tests drive the same loop with a CPU backend to check admission and
accounting.
"""
from __future__ import annotations

import bisect
import collections
import heapq
import time
from dataclasses import dataclass, field

import numpy as np


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
    lane: int = 0


@dataclass
class ServeStats:
    completed: int = 0
    events: int = 0
    wall_s: float = 0.0
    max_active: int = 0
    mean_active: float = 0.0
    max_bytes: int = 0
    ticks: int = 0
    lanes: int = 1
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
            "max_hbm_bytes": self.max_bytes, "ticks": self.ticks, "lanes": self.lanes,
        }


def chain_estimate(problem: dict) -> float:
    """Expected events per step of the tissue's busiest cell: the propensity
    of an average voxel (mass action at the mean initial counts, diffusion
    at degree 3) times the largest cell's voxel count times dt."""
    p = problem
    S = int(p["n_species"])
    x = np.asarray(p["init_counts"], np.float64).reshape(-1, S).mean(axis=0)
    a = 0.0
    for r, (ra, rb) in enumerate(np.asarray(p["reactants"], np.int64).reshape(-1, 2)):
        if ra < 0 and rb < 0:
            a += p["rates"][r]
        elif ra < 0 or rb < 0:
            a += p["rates"][r] * x[max(ra, rb)]
        elif ra == rb:
            a += p["rates"][r] * x[ra] * (x[ra] - 1.0) * 0.5
        else:
            a += p["rates"][r] * x[ra] * x[rb]
    a += 3.0 * float(np.dot(np.asarray(p["diffusion"], np.float64), x))
    vmax = int(np.max(np.asarray(p["mesh_w"], np.int64) * np.asarray(p["mesh_h"], np.int64)))
    return a * vmax * float(p["dt"])


class Server:
    """Continuous-batching loop over `lanes` independent lanes.

    backend: object with lanes (int), required_bytes(problem),
      create(problem, lane), step(lane, handles, dt, n, finishing) (advance
      all handles by n steps, asynchronously allowed; `finishing` are the
      handles whose last step this is, whose totals events() will report),
      busy(lane) (the lane's last step still running), sync(lane),
      events(handle), read(handle), free(lane, handle).
    max_bytes: HBM budget for resident tissues; max_active: slot count over
    all lanes; quantum: steps per tick.  Requests go to lanes by the rank of
    chain_estimate among the requests seen so far (one lane: all).
    """

    def __init__(self, backend, max_bytes: int, max_active: int = 4096, quantum: int = 10,
                 clock=time.perf_counter, keep_results: bool = False):
        self.backend = backend
        self.max_bytes = int(max_bytes)
        self.max_active = int(max_active)
        self.quantum = int(quantum)
        self.clock = clock
        self.keep_results = keep_results
        self.lanes = max(1, int(getattr(backend, "lanes", 1)))
        self._seen: list = []

    def _route(self, r: Request) -> int:
        if self.lanes == 1:
            return 0
        e = chain_estimate(r.problem)
        rank = bisect.bisect_left(self._seen, e) / max(len(self._seen), 1)
        bisect.insort(self._seen, e)
        return min(self.lanes - 1, int(rank * self.lanes))

    def run(self, requests, real_time: bool = True) -> tuple[ServeStats, list]:
        """Serve `requests` (sorted by arrival).  With real_time, arrivals are
        replayed against the wall clock (a request cannot be admitted before
        its arrival time); otherwise the clock is virtual: it advances by the
        measured time of each pass of the loop and jumps over idle gaps."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        K = self.lanes
        waiting = [[] for _ in range(K)]   # per lane: (arrival, rid, req)
        active = [[] for _ in range(K)]
        inflight = [0] * K                 # steps of the running tick (0: idle)
        done: list[Request] = []
        st = ServeStats(lanes=K)
        used = 0
        n_active = 0
        t0 = self.clock()
        vt = 0.0
        last = t0
        active_sum = 0

        def now():
            return (self.clock() - t0) if real_time else vt

        while pending or any(waiting) or n_active:
            if not real_time:
                c = self.clock()
                vt += c - last
                last = c
            while pending and pending[0].arrival <= now():
                r = pending.popleft()
                r.lane = self._route(r)
                heapq.heappush(waiting[r.lane], (r.arrival, r.rid, r))
            progressed = False
            for L in range(K):
                if inflight[L]:
                    if self.backend.busy(L):
                        continue
                    # the lane's tick has finished: account for it
                    q = inflight[L]
                    inflight[L] = 0
                    progressed = True
                    end = now()
                    still = []
                    for r in active[L]:
                        r.steps_done += q
                        if r.steps_done >= r.n_steps:
                            r.events = self.backend.events(r.handle)
                            if self.keep_results:
                                r.result = self.backend.read(r.handle)
                            self.backend.free(L, r.handle)
                            r.handle = None
                            used -= r.bytes
                            n_active -= 1
                            r.finished = end
                            st.completed += 1
                            st.events += r.events
                            st.latencies.append(r.finished - r.arrival)
                            st.queue_waits.append(r.admitted - r.arrival)
                            done.append(r)
                        else:
                            still.append(r)
                    active[L] = still
                # admission into this lane: oldest first, by slots and HBM
                while waiting[L] and n_active < self.max_active:
                    r = waiting[L][0][2]
                    need = self.backend.required_bytes(r.problem)
                    if need > self.max_bytes:
                        raise ValueError(f"request {r.rid} needs {need} B, over the whole budget")
                    if used + need > self.max_bytes:
                        break
                    heapq.heappop(waiting[L])
                    r.bytes = need
                    r.handle = self.backend.create(r.problem, L)
                    r.admitted = now()
                    used += need
                    n_active += 1
                    active[L].append(r)
                    progressed = True
                if active[L]:
                    q = min([self.quantum] + [r.n_steps - r.steps_done for r in active[L]])
                    by_dt = collections.defaultdict(list)
                    ending = collections.defaultdict(list)
                    for r in active[L]:
                        by_dt[r.problem["dt"]].append(r.handle)
                        if r.steps_done + q >= r.n_steps:
                            ending[r.problem["dt"]].append(r.handle)
                    for d, hs in by_dt.items():
                        self.backend.step(L, hs, d, q, ending[d])
                    inflight[L] = q
                    st.ticks += 1
                    active_sum += n_active
                    progressed = True
            st.max_active = max(st.max_active, n_active)
            st.max_bytes = max(st.max_bytes, used)
            if progressed:
                continue
            if not any(inflight):
                # idle: wait for the next arrival
                if not pending:
                    break
                if real_time:
                    delay = pending[0].arrival - now()
                    if delay > 0:
                        time.sleep(min(delay, 0.05))
                else:
                    vt = max(vt, pending[0].arrival)
                    last = self.clock()
            else:
                # the device is busy: wait a little for a lane to finish
                time.sleep(2e-4)
        st.wall_s = now()
        st.mean_active = active_sum / st.ticks if st.ticks else 0.0
        return st, done


class GpuBackend:
    """The C-ABI library as a serving backend: one Tissue per request (its
    own device buffer), per lane one stream and one Batch per distinct
    active set, rebuilt only when the set changes.

    Each lane needs a hardware queue of its own: HIP maps streams onto
    GPU_MAX_HW_QUEUES queues (4 by default, set before the runtime starts),
    and a lane sharing a queue waits behind the other lane's kernels in
    every synchronisation (creation, batch rebuild), which the loop cannot
    hide.  Use a queue count of at least the lanes plus two."""

    def __init__(self, device="cuda:0", lanes: int = 4, graph_chunk: int = 0,
                 persistent: bool = False, max_slots: int = 8192, regroup: int = 2):
        import os
        import warnings

        import torch

        from . import tissue as T
        self.T = T
        self.torch = torch
        self.device = device
        self.lanes = int(lanes)
        if self.lanes > 1 and int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < self.lanes + 2:
            warnings.warn(f"{self.lanes} serving lanes with GPU_MAX_HW_QUEUES="
                          f"{os.environ.get('GPU_MAX_HW_QUEUES', '4 (default)')}: lanes may share "
                          "hardware queues and wait on each other", RuntimeWarning)
        # default priority on every stream
        self.streams = [torch.cuda.Stream(device=device) for _ in range(self.lanes)]
        self.graph_chunk = graph_chunk
        # one workgroup per work item, so that the lanes' kernels share the
        # compute units as their workgroups retire (a persistent grid holds
        # every CU until its slowest item is done)
        self.persistent = bool(persistent)
        self.regroup = int(regroup)  # the load-ordered regroup before compact launches
        self._batch = [None] * self.lanes
        self._key = [None] * self.lanes
        self._done = [None] * self.lanes
        self._bytes = {}
        # pinned host slots for the statistics blocks copied at the end of a
        # request's last tick (no blocking read in the serving loop)
        B = T.STATS_BLOCK_BYTES
        self._stats_host = torch.empty(max_slots * B, dtype=torch.uint8, pin_memory=True)
        self._free_slots = list(range(max_slots - 1, -1, -1))
        self._slot = {}

    def required_bytes(self, problem):
        k = id(problem)
        if k not in self._bytes:
            self._bytes[k] = self.T.required_bytes(problem) + 256
        return self._bytes[k]

    def create(self, problem, lane):
        self._bytes.pop(id(problem), None)
        with self.torch.cuda.stream(self.streams[lane]):
            t = self.T.Tissue(problem, device=self.device, stream=self.streams[lane])
        self._slot[id(t)] = self._free_slots.pop()
        return t

    def _slot_ptr(self, h):
        return self._stats_host.data_ptr() + self._slot[id(h)] * self.T.STATS_BLOCK_BYTES

    def step(self, lane, handles, dt, n, finishing=()):
        key = tuple(id(h) for h in handles)
        if key != self._key[lane]:
            if self._batch[lane] is not None:
                self._batch[lane].close()
            self._batch[lane] = self.T.Batch(handles, device=self.device, stream=self.streams[lane])
            self._batch[lane].set_graph_chunk(self.graph_chunk)
            self._batch[lane].set_launch(self.persistent, 0)
            if self.regroup != 2:
                self._batch[lane].set_regroup(self.regroup)
            self._key[lane] = key
        self._batch[lane].step(dt, n)
        for h in finishing:
            h.stats_enqueue(self._slot_ptr(h))
        ev = self.torch.cuda.Event()
        ev.record(self.streams[lane])
        self._done[lane] = ev

    def busy(self, lane):
        ev = self._done[lane]
        return ev is not None and not ev.query()

    def sync(self, lane):
        if self._batch[lane] is not None:
            self._batch[lane].sync()

    def events(self, h):
        # the block copied at the end of the request's last tick (the lane's
        # completion event has passed it)
        st = h.stats_decode(self._slot_ptr(h))
        return st["chi_events"] + st["s_events"]

    def read(self, h):
        return h.read_counts()

    def free(self, lane, h):
        if self._batch[lane] is not None:
            self._batch[lane].close()
            self._batch[lane], self._key[lane] = None, None
        h.close()
        h.buffer = None
        self._free_slots.append(self._slot.pop(id(h)))


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
