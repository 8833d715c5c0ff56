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


# submission results, the library's codes (include/tissue.h)
OK, EINVAL, EBUSY = 0, -1, -5


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
    status: str = "pending"        # then "waiting", "active", and at the end
                                   # "done", "cancelled", "failed" or "rejected"
    error: str = ""
    cancel_requested: bool = False


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
    cancelled: int = 0
    failed: int = 0
    rejected: int = 0
    busy_retries: int = 0
    budget_bytes: int = 0
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
            "max_hbm_bytes": self.max_bytes, "budget_bytes": self.budget_bytes,
            "ticks": self.ticks, "lanes": self.lanes,
            "cancelled": self.cancelled, "failed": self.failed, "rejected": self.rejected,
            "busy_retries": self.busy_retries,
        }


def chain_estimate(problem: dict) -> float:
    """Expected events per step of the tissue's busiest cell: the propensity
    of an average voxel (mass action at the mean initial counts, diffusion
    at degree 3) times the largest cell's voxel count times dt."""
    p = problem
    S = int(p["n_species"])
    c = np.asarray(p["init_counts"]).reshape(-1, S)
    # (per-species column sums: much faster than a strided reduction over axis 0)
    x = np.array([float(c[:, s].sum(dtype=np.int64)) for s in range(S)]) / max(c.shape[0], 1)
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
      events(handle), read(handle), and retire(lane, handles) (release
      finished or abandoned requests; free(lane, handle) for one at a time
      where there is no retire), and optionally free_bytes() (device memory
      free now).
    max_bytes: HBM budget for resident tissues; None: the backend's free
      memory at start minus margin_bytes.  max_active: slot count over all
      lanes; quantum: steps per tick.  max_waiting: bound on admitted-but-
      waiting requests, beyond which submit() answers EBUSY (None: no
      bound).  tick_deadline_s: a lane's tick still running after this long
      fails the requests in it (they are released when the tick ends; the
      loop goes on; None: no deadline).  Requests go to lanes by the rank
      of chain_estimate among the requests seen so far (one lane: all).
    """

    def __init__(self, backend, max_bytes=None, max_active: int = 4096, quantum: int = 10,
                 clock=time.perf_counter, keep_results: bool = False, max_waiting=None,
                 tick_deadline_s=None, margin_bytes: int = 1 << 30, sleep=time.sleep):
        self.backend = backend
        if max_bytes is None:
            max_bytes = max(0, int(backend.free_bytes()) - int(margin_bytes))
        self.max_bytes = int(max_bytes)
        self.max_active = int(max_active)
        self.quantum = int(quantum)
        self.clock = clock
        self.sleep = sleep
        self.keep_results = keep_results
        self.max_waiting = max_waiting
        self.tick_deadline_s = tick_deadline_s
        self.lanes = max(1, int(getattr(backend, "lanes", 1)))
        self._seen: list = []
        self._reset()

    def _reset(self):
        K = self.lanes
        self.waiting = [[] for _ in range(K)]   # per lane: (arrival, rid, req)
        self.active = [[] for _ in range(K)]
        self.by_id = {}
        self.n_waiting = 0
        self.done: list[Request] = []
        self.st = ServeStats(lanes=K, budget_bytes=self.max_bytes)
        self.used = 0
        self.n_active = 0

    def _route(self, r: Request) -> int:
        if self.lanes == 1:
            return 0
        e = chain_estimate(r.problem)
        rank = bisect.bisect_left(self._seen, e) / max(len(self._seen), 1)
        bisect.insort(self._seen, e)
        return min(self.lanes - 1, int(rank * self.lanes))

    def _end(self, r: Request, status: str, when: float, error: str = ""):
        r.status, r.error, r.finished = status, error, when
        if status == "cancelled":
            self.st.cancelled += 1
        elif status == "failed":
            self.st.failed += 1
        elif status == "rejected":
            self.st.rejected += 1
        self.done.append(r)

    def submit(self, r: Request, now: float = 0.0) -> int:
        """Queue a request for admission.  EINVAL: it can never fit the budget
        (ended as "rejected"); EBUSY: the waiting queue is full -- retry
        later; OK: queued."""
        need = self.backend.required_bytes(r.problem)
        if need > self.max_bytes:
            self._end(r, "rejected", now, f"needs {need} B, over the whole budget of {self.max_bytes} B")
            return EINVAL
        if self.max_waiting is not None and self.n_waiting >= self.max_waiting:
            return EBUSY
        r.bytes = need
        r.lane = self._route(r)
        r.status = "waiting"
        heapq.heappush(self.waiting[r.lane], (r.arrival, r.rid, r))
        self.n_waiting += 1
        self.by_id[r.rid] = r
        return OK

    def cancel(self, rid: int, now: float = 0.0) -> bool:
        """Cancel a submitted request: a waiting one leaves the queue at
        once, an active one is released when its lane's tick ends."""
        r = self.by_id.get(rid)
        if r is None or r.status not in ("waiting", "active"):
            return False
        if r.status == "waiting":
            self.waiting[r.lane] = [e for e in self.waiting[r.lane] if e[2] is not r]
            heapq.heapify(self.waiting[r.lane])
            self.n_waiting -= 1
            self._end(r, "cancelled", now)
        else:
            r.cancel_requested = True
        return True

    def _retire(self, L: int, rs):
        if not rs:
            return
        hs = [r.handle for r in rs]
        if hasattr(self.backend, "retire"):
            self.backend.retire(L, hs)
        else:
            for h in hs:
                self.backend.free(L, h)
        for r in rs:
            r.handle = None
            self.used -= r.bytes
            self.n_active -= 1

    def run(self, requests, real_time: bool = True, cancels=(), busy_retry_s: float = 0.005):
        """Serve `requests` (by arrival time).  With real_time, arrivals are
        replayed against the clock (a request cannot be admitted before its
        arrival time); otherwise the clock is virtual: it advances by the
        measured time of each pass of the loop and jumps over idle gaps.
        cancels: (time, rid) pairs, each cancelling that request at that
        time.  A submission answered EBUSY is tried again busy_retry_s
        later (its latency still counts from its arrival)."""
        self._reset()
        every = {r.rid: r for r in requests}
        pending = sorted(((r.arrival, r.rid, r) for r in requests), key=lambda e: e[:2])
        heapq.heapify(pending)
        cancel_q = sorted(cancels)
        K = self.lanes
        inflight = [0] * K                 # steps of the running tick (0: idle)
        started = [0.0] * K                # when it was launched
        st = self.st
        t0 = self.clock()
        vt = 0.0
        last = t0
        active_sum = 0

        def now():
            return (self.clock() - t0) if real_time else vt

        while pending or self.n_waiting or self.n_active or any(inflight):
            if not real_time:
                c = self.clock()
                vt += c - last
                last = c
            while pending and pending[0][0] <= now():
                when, rid, r = heapq.heappop(pending)
                if r.cancel_requested:  # cancelled before it was submitted
                    self._end(r, "cancelled", now())
                    continue
                rc = self.submit(r, now())
                if rc == EBUSY:
                    st.busy_retries += 1
                    heapq.heappush(pending, (now() + busy_retry_s, rid, r))
            while cancel_q and cancel_q[0][0] <= now():
                _, rid = cancel_q.pop(0)
                if not self.cancel(rid, now()) and rid in every and every[rid].status == "pending":
                    every[rid].cancel_requested = True
            progressed = False
            for L in range(K):
                if inflight[L]:
                    if self.backend.busy(L):
                        if (self.tick_deadline_s is not None and
                                now() - started[L] > self.tick_deadline_s):
                            for r in self.active[L]:
                                if r.status == "active":
                                    r.status = "failing"
                                    r.error = f"tick over its deadline of {self.tick_deadline_s} s"
                        continue
                    # the lane's tick has finished: account for it
                    q = inflight[L]
                    inflight[L] = 0
                    progressed = True
                    end = now()
                    still, leave = [], []
                    for r in self.active[L]:
                        r.steps_done += q
                        if r.status == "failing":
                            leave.append(r)
                            self._end(r, "failed", end, r.error)
                        elif r.cancel_requested:
                            leave.append(r)
                            self._end(r, "cancelled", end)
                        elif r.steps_done >= r.n_steps:
                            r.events = self.backend.events(r.handle)
                            if self.keep_results:
                                r.result = self.backend.read(r.handle)
                            leave.append(r)
                            self._end(r, "done", end)
                            st.completed += 1
                            st.events += r.events
                            st.latencies.append(r.finished - r.arrival)
                            st.queue_waits.append(r.admitted - r.arrival)
                        else:
                            still.append(r)
                    self._retire(L, leave)
                    self.active[L] = still
                # admission into this lane: oldest first, by slots and HBM
                while self.waiting[L] and self.n_active < self.max_active:
                    r = self.waiting[L][0][2]
                    if self.used + r.bytes > self.max_bytes:
                        break
                    heapq.heappop(self.waiting[L])
                    self.n_waiting -= 1
                    r.handle = self.backend.create(r.problem, L)
                    r.admitted = now()
                    r.status = "active"
                    self.used += r.bytes
                    self.n_active += 1
                    self.active[L].append(r)
                    progressed = True
                if self.active[L]:
                    q = min([self.quantum] + [r.n_steps - r.steps_done for r in self.active[L]])
                    by_dt = collections.defaultdict(list)
                    ending = collections.defaultdict(list)
                    for r in self.active[L]:
                        by_dt[r.problem["dt"]].append(r.handle)
                        if r.steps_done + q >= r.n_steps:
                            ending[r.problem["dt"]].append(r.handle)
                    for d, hs in by_dt.items():
                        self.backend.step(L, hs, d, q, ending[d])
                    inflight[L] = q
                    started[L] = now()
                    st.ticks += 1
                    active_sum += self.n_active
                    progressed = True
            st.max_active = max(st.max_active, self.n_active)
            st.max_bytes = max(st.max_bytes, self.used)
            if progressed:
                continue
            if not any(inflight):
                # idle: wait for the next arrival
                if not pending:
                    if not self.n_waiting:
                        break
                    continue
                if real_time:
                    delay = pending[0][0] - now()
                    if delay > 0:
                        self.sleep(min(delay, 0.05))
                else:
                    vt = max(vt, pending[0][0])
                    last = self.clock()
            else:
                # the device is busy: wait a little for a lane to finish
                self.sleep(2e-4)
        st.wall_s = now()
        st.mean_active = active_sum / st.ticks if st.ticks else 0.0
        return st, self.done


class GpuBackend:
    """The C-ABI library as a serving backend: one Tissue per request (its
    own device buffer), per lane one stream and one Batch whose members are
    replaced in place (tissue_batch_set_members: the work lists are planned
    again and copied on the lane's stream, with no host synchronisation and
    no new batch) as requests are admitted and retired.  A lane's batch is
    created at its first admission with a work-list buffer of
    `lane_capacity_bytes`, and made again, larger, only when a member set
    outgrows it (set_members answers EBUSY).

    Each lane needs a hardware queue of its own: HIP maps streams onto
    GPU_MAX_HW_QUEUES queues (4 by default, set before the runtime starts),
    and a lane sharing a queue waits behind the other lane's kernels in
    every synchronisation (creation), which the loop cannot hide.  Use a
    queue count of at least the lanes plus two."""

    def __init__(self, device="cuda:0", lanes: int = 4, graph_chunk: int = 0,
                 persistent: bool = False, max_slots: int = 8192, regroup: int = 2,
                 lane_capacity_bytes: int = 32 << 20):
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
        self.capacity = int(lane_capacity_bytes)
        self._batch = [None] * self.lanes
        self._members = [[] for _ in range(self.lanes)]
        self._done = [None] * self.lanes
        self._bytes = {}
        self.rebuilds = 0
        # pinned host slots for the statistics blocks copied at the end of a
        # request's last tick (no blocking read in the serving loop)
        B = T.STATS_BLOCK_BYTES
        self._stats_host = torch.empty(max_slots * B, dtype=torch.uint8, pin_memory=True)
        self._free_slots = list(range(max_slots - 1, -1, -1))
        self._slot = {}

    def free_bytes(self):
        return self.torch.cuda.mem_get_info(self.device)[0]

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

    def _set_members(self, lane, handles):
        """The lane's batch with exactly these members (made at first use,
        made again larger when they outgrow its buffer)."""
        handles = list(handles)
        if [id(h) for h in handles] == [id(h) for h in self._members[lane]]:
            return
        b = self._batch[lane]
        if b is not None:
            try:
                b.set_members(handles)
                self._members[lane] = handles
                return
            except self.T.TissueError as e:
                if e.code != self.T.EBUSY:
                    raise
                b.set_members([])
                b.close()
                self._batch[lane] = None
                self.capacity *= 2
        if not handles:
            self._members[lane] = []
            return
        b = self.T.Batch(handles, device=self.device, stream=self.streams[lane],
                         capacity_bytes=self.capacity)
        b.set_graph_chunk(self.graph_chunk)
        b.set_launch(self.persistent, 0)
        if self.regroup != 2:
            b.set_regroup(self.regroup)
        self._batch[lane] = b
        self._members[lane] = handles
        self.rebuilds += 1

    def step(self, lane, handles, dt, n, finishing=()):
        self._set_members(lane, handles)
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

    def retire(self, lane, handles):
        """Release finished or abandoned requests: out of the lane's batch
        first (a member cannot be destroyed), then destroyed."""
        gone = {id(h) for h in handles}
        self._set_members(lane, [h for h in self._members[lane] if id(h) not in gone])
        for h in handles:
            h.close()
            h.buffer = None
            self._free_slots.append(self._slot.pop(id(h)))

    def free(self, lane, h):
        self.retire(lane, [h])


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
