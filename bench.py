"""Benchmark: SSA events/s of the split multicellular simulation on one MI355X.

Workload (default): the 64x64 hex tissue of 4096 cells, 4x4 voxels per cell,
the 5-species Notch-Delta network with 9 internal reactions + the trans
reaction, diffusion 1.0, dt = 0.05, T = 100 (2000 splitting steps), seeded
synthetic inputs.  One benchmark step = restart the resident tissue from its
initial counts as a new simulation (sim_id = step index) and advance it over
the whole horizon T (tissue_step(dt, 2000), replayed from captured HIP
graphs).  value = (chi + S events) / wall time of the K timed steps.

Also reported: the chi kernel's roofline fraction -- algorithmic lane
operations per event (counted per leaf class) times events per launch over
the live launch time (HIP events around every launch of one extra
simulation over the same horizon, launched eagerly on the tissue's stream),
or over the timed steps' wall time where a step forks several classes'
launches -- with VALU busy, issued lane-slots per event and HBM bytes from
the committed rocprofv3 counter figures of the same sources; the CPU FP64
oracle's rate on a bounded sample on the host cores; the tiny plain
workload (latency per simulation and per step); the batched form (512
tissues in one batch, with its own roofline) and the serving loop
(Poisson arrivals, continuous batching, p50/p99 latency).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--leg all|plain|tiny|uneven|batched|serving|dt|notch|multifidelity|large]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HIP maps streams onto GPU_MAX_HW_QUEUES hardware queues (4 by default);
# the serving leg's lanes each need a queue of their own, or a lane's
# synchronisation waits behind another lane's kernels.  Set before the HIP
# runtime starts (torch is imported later).
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

METRIC = "SSA events/sec on 1 MI355X (batched vs plain); p50/p99 sim latency"

# Algorithmic VALU work per accepted chi event, in full-rate lane-operation
# equivalents (a quarter-rate instruction counts 4): a fixed part (Philox4x32-10
# 120, two uniforms 12, plog 40, the clock 15, r = U2 a0 1, the apply 6), per
# channel slot of a voxel the scan (7) and the refolds of the two changed
# voxels (8), per tree level the descent (5) and the two ancestor paths (2).
# The 5-species network has 14 channel slots (9 reactions, 5 diffusing
# species): 432 on cells of 16 leaves.  Derivation in the design notes.
OPS_FIXED, OPS_PER_CHANNEL, OPS_PER_LEVEL = 194, 15, 7
OPS_PER_S_EVENT = 289


def ops_per_chi_event(leaves: int, channels: int = 14) -> float:
    return OPS_FIXED + OPS_PER_CHANNEL * channels + OPS_PER_LEVEL * math.log2(max(leaves, 1))


def ops_per_chi_event_of(p) -> float:
    """Weighted over the tissue's leaf-count classes by their share of the
    voxels (events per voxel are alike across the classes)."""
    import numpy as np
    V = np.asarray(p["mesh_w"], np.int64) * np.asarray(p["mesh_h"], np.int64)
    P = 2.0 ** np.ceil(np.log2(np.maximum(V, 1)))
    ch = int(p["n_reactions"]) + int((np.asarray(p["diffusion"]) > 0).sum())
    return float(np.sum(V * (OPS_FIXED + OPS_PER_CHANNEL * ch + OPS_PER_LEVEL * np.log2(P))) / V.sum())


# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-ops/s
N_SIMD, CLOCK_HZ = 256 * 4, 2.4e9
PEAK_LANE_OPS = N_SIMD * 16 * CLOCK_HZ
PEAK_HBM = 8.0e12

# Counter figures of each leg's chi kernels from rocprofv3 runs of this
# script (profiles/), per dispatch: the kernel-trace duration and the SQ
# counters of the same run, FETCH_SIZE and WRITE_SIZE (KiB; each pass also
# carries the SQ counters and the duration).  FETCH_SIZE and WRITE_SIZE are
# scaled by what they read for a plain 256 MiB device copy (FETCH 131085 KiB,
# WRITE 262144 KiB for 262144 KiB moved each way).  chi_events_per_step is
# that run's own count (chi events over the steps it ran, from its bench
# line).  The figures hold for the kernel sources whose digest is recorded;
# any change to those sources makes them null until the counters are taken
# again.
FETCH_SCALE = 262144.0 / 131085.0
WRITE_SCALE = 262144.0 / 262144.0
COUNTERS = {
    "plain": {
        "digest": "5ae5c01a1874fef8f7ed5afd81ee266678ffe815",
        "profile": "profiles/chi_row_plain_hex64x64_4x4.md",
        "chi_events_per_step": 744850.5,
        "kernels": {
            "tissue_chi_row": {
                "dispatches_per_step": 1.0,
                "avg_us": 168.637,
                "sq_insts_valu": 46678900.0,
                "fetch_kib": 934.241,
                "write_kib": 1376.0
            }
        }
    },
    "batched": {
        "digest": "5ae5c01a1874fef8f7ed5afd81ee266678ffe815",
        "profile": "profiles/chi_lane16_batched_512_tissues.md",
        "chi_events_per_step": 1298376166.0,
        "kernels": {
            "tissue_chi_lane16": {
                "dispatches_per_step": 1.0,
                "avg_us": 19870.414,
                "sq_insts_valu": 10691100000.0,
                "fetch_kib": 652282.0,
                "write_kib": 1058540.0
            }
        }
    },
    "uneven": {
        "digest": "5ae5c01a1874fef8f7ed5afd81ee266678ffe815",
        "profile": "profiles/chi_classes_uneven_hex256x256.md",
        "chi_events_per_step": 22521846.2,
        "kernels": {
            "tissue_chi_row64": {
                "dispatches_per_step": 1.0,
                "avg_us": 1231.577,
                "sq_insts_valu": 326999000.0,
                "fetch_kib": 876.96,
                "write_kib": 1222.38
            },
            "tissue_chi_lane16x4": {
                "dispatches_per_step": 1.0,
                "avg_us": 1513.735,
                "sq_insts_valu": 91578300.0,
                "fetch_kib": 2410.94,
                "write_kib": 3341.36
            },
            "tissue_chi_lane16x2": {
                "dispatches_per_step": 1.0,
                "avg_us": 1036.49,
                "sq_insts_valu": 141730000.0,
                "fetch_kib": 7338.0,
                "write_kib": 10512.1
            },
            "tissue_chi_lane16": {
                "dispatches_per_step": 1.0,
                "avg_us": 535.785,
                "sq_insts_valu": 74519500.0,
                "fetch_kib": 8808.59,
                "write_kib": 11674.4
            },
            "tissue_chi_lane": {
                "dispatches_per_step": 3.0,
                "avg_us": 9.303,
                "sq_insts_valu": 27655.0,
                "fetch_kib": 29.7576,
                "write_kib": 16.0938
            }
        }
    }
}


def kernel_source_digest() -> str:
    """SHA-1 over the library's device and launch sources (csrc/)."""
    d = os.path.join(ROOT, "paper_1806_10889_amd", "csrc")
    h = hashlib.sha1()
    for name in sorted(os.listdir(d)):
        if name.endswith((".h", ".hip", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def counter_figures(leg: str, kernels=None, live_s_per_step=None):
    """VALU busy, issued lane-slots per event and HBM bytes of the leg's chi
    kernels (per step: dispatches_per_step of each, default one) from the
    committed counter figures, or None when they were taken on other
    sources.  VALU busy =
    SQ_INSTS_VALU x 4 cycles / (SIMDs x the dispatch's own duration in that
    run x clock); lane-slots per event = SQ_INSTS_VALU x 64 / chi events
    per step; HBM fraction = the scaled FETCH + WRITE bytes over the live
    time per step (or the counter run's duration) / 8 TB/s; valu_busy_live =
    the same instructions over the live time per step."""
    rec = COUNTERS.get(leg)
    if not rec or rec["digest"] != kernel_source_digest():
        return None
    kernels = sorted(rec["kernels"]) if kernels is None else kernels
    ks = [rec["kernels"][k] for k in kernels if k in rec["kernels"]]
    if not kernels or len(ks) != len(kernels):
        return None
    per = [k.get("dispatches_per_step", 1) for k in ks]
    valu = sum(n * k["sq_insts_valu"] for n, k in zip(per, ks))
    dur = sum(n * k["avg_us"] for n, k in zip(per, ks)) * 1e-6
    traffic = 1024.0 * sum(n * (k["fetch_kib"] * FETCH_SCALE + k["write_kib"] * WRITE_SCALE)
                           for n, k in zip(per, ks))
    t = live_s_per_step or dur
    return {"kernels": list(kernels), "valu_busy": valu * 4.0 / (N_SIMD * dur * CLOCK_HZ),
            "valu_busy_live": valu * 4.0 / (N_SIMD * t * CLOCK_HZ),
            "issued_lane_slots_per_event": valu * 64.0 / rec["chi_events_per_step"],
            "counter_run_us_per_step": dur * 1e6, "traffic": traffic,
            "hbm_frac": traffic / t / PEAK_HBM, "profile": rec["profile"]}


def chi_kernel_name(mode: int, jit: bool, leaves: int = 16, refill: int = 0) -> str:
    base = {0: "lane", 1: "row", 3: "lane16", 4: "row"}.get(mode, "unknown")
    if base == "lane16" and leaves > 16:
        base += f"x{leaves // 16}"  # the compact layout with 2 or 4 lanes per cell
    elif base == "lane16" and refill and jit:
        base += "r"  # one lane per cell, lanes refilled
    if base == "row" and jit and (leaves > 16 or mode == 4):
        base += str(max(leaves, 32) if mode == 4 else leaves)
    return f"tissue_chi_{base}" if jit else f"chi_{base}_kernel"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pct(a, q):
    a = sorted(a)
    if not a:
        return None
    k = (len(a) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return a[lo] + (a[hi] - a[lo]) * (k - lo)


def run_single(args, torch, T, p, leg, sims, warmup):
    """One resident tissue: `sims` timed simulations over the problem's whole
    horizon (restart with a new sim_id, then tissue_step), after `warmup`
    untimed ones; then the eager roofline pass."""
    stream = torch.cuda.current_stream()
    t = T.Tissue(p, device="cuda:0", stream=stream)
    t.set_regroup(args.regroup)
    if args.refill >= 0:
        t.set_refill(args.refill)
    dt, n = p["dt"], p["n_steps"]
    if args.launch:
        mode, persistent, wpc, chunk = (int(v) for v in args.launch.split(","))
        t.set_chi_mode(mode)
        t.set_launch(bool(persistent), wpc)
        t.set_graph_chunk(chunk)
        tuned = {"config": dict(chi_mode=mode, persistent=persistent, wpc=wpc, graph_chunk=chunk)}
    elif args.no_tune:
        t.set_launch(True, 0)
        t.set_graph_chunk(args.graph_chunk)
        tuned = None
    else:
        from paper_1806_10889_amd import autotune
        tuned = autotune.tune([p], dt, steps=min(50, n), reps=2, target=t, log=log)
        log(f"autotuned launch: {tuned['config']}")
    basis = {"chi_events": 0, "steps": 0}  # every chi step this leg runs after tuning

    def one(k):
        t.restart(sim_id=k, start_step=0)
        t.step(dt, n)
        st = t.stats()  # synchronises the stream
        basis["chi_events"] += st["chi_events"]
        basis["steps"] += n
        return st["chi_events"] + st["s_events"], st

    for w in range(warmup):
        one(1000 + w)
        log(f"{leg}: warmup {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    lat, events, chi_ev, s_ev = [], 0, 0, 0
    t0 = time.perf_counter()
    for k in range(sims):
        a = time.perf_counter()
        ev, st = one(k)
        lat.append(time.perf_counter() - a)
        events += ev
        chi_ev += st["chi_events"]
        s_ev += st["s_events"]
        log(f"{leg}: simulation {k + 1}/{sims}: {ev} events in {lat[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # roofline pass: one more simulation over the same horizon, launched
    # eagerly with every kernel bracketed by HIP events on the tissue's stream
    ops = ops_per_chi_event_of(p)
    t.restart(sim_id=sims + 7, start_step=0)
    rsteps = min(n, args.roofline_steps) if args.roofline_steps > 0 else n
    tm = t.step_timed(dt, rsteps)
    st = t.stats()
    basis["chi_events"] += st["chi_events"]
    basis["steps"] += rsteps
    chi_per_launch = st["chi_events"] / max(tm["chi_launches"], 1)
    chi_avg_ms = tm["chi_ms"] / max(tm["chi_launches"], 1)
    s_avg_ms = tm["s_ms"] / max(tm["s_launches"], 1)
    kernel = chi_kernel_name(tm["chi_kernel"], bool(st["jit"]), tm["chi_leaves"], tm["chi_refill"])
    launches_per_step = tm["chi_launches"] / max(rsteps, 1)
    # the timed run: chi events x algorithmic operations over its wall time
    timed = {"basis": "the timed simulations' chi events over their whole wall time (every "
                      "kernel of a step, launch gaps included)",
             "achieved": chi_ev * ops / elapsed / 1e12, "frac": chi_ev * ops / elapsed / PEAK_LANE_OPS}
    if launches_per_step <= 1.0 + 1e-9:
        # one chi launch per step: the kernel's own rate from its live launch times
        achieved = chi_per_launch * ops / (chi_avg_ms * 1e-3)
        cnt = counter_figures(leg, [kernel], live_s_per_step=chi_avg_ms * 1e-3)
        roof = {"bound": "alu", "kernel": kernel,
                "basis": "HIP events around every chi launch of one eager simulation over the horizon",
                "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
                "frac": achieved / PEAK_LANE_OPS, "avg_launch_ms": chi_avg_ms,
                "events_per_launch": chi_per_launch}
    else:
        # several classes' launches per step, run as parallel graph branches in
        # the timed run: the rate of the timed steps themselves
        cnt = counter_figures(leg, None, live_s_per_step=elapsed / max(sims * n, 1))
        roof = {"bound": "alu", "kernel": "every chi launch of a step (forked graph branches)",
                "basis": timed["basis"], "achieved": timed["achieved"],
                "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s", "frac": timed["frac"],
                "eager_dominant_kernel": kernel,
                "eager_avg_launch_ms": chi_avg_ms, "events_per_step": st["chi_events"] / max(rsteps, 1)}
    roof.update({"ops_per_event": ops, "traffic": cnt["traffic"] if cnt else None,
                 "hbm_frac": cnt["hbm_frac"] if cnt else None, "counters": cnt,
                 "timed_run": timed, "s_kernel_avg_ms": s_avg_ms,
                 "chi_share_of_kernel_time": tm["chi_ms"] / max(tm["chi_ms"] + tm["s_ms"], 1e-12),
                 "counter_basis": dict(basis)})
    res = dict(p=p, value=events / elapsed, elapsed=elapsed, lat=lat, chi=chi_ev, s=s_ev,
               roofline=roof, timing=tm, tuned=tuned, jit=bool(t.stats()["jit"]))
    cfg = (tuned or {}).get("config")
    t.close()
    if args.chain_steps > 0:
        res["roofline"]["event_chains"], more = event_chains(args, T, p, cfg)
        for k in ("chi_events", "steps"):
            res["roofline"]["counter_basis"][k] += more[k]
    return res


def event_chains(args, T, p, cfg):
    """The latency side of the chi launch: each cell's events in a step form
    one dependent chain, and a launch lasts as long as its busiest cell's
    chain.  A traced simulation over the first chain_steps steps (by default
    the whole horizon; eager, HIP events around every launch) gives, per
    step, the busiest cell's and the mean cell's events, and the time per
    event along the busiest chain."""
    import numpy as np
    n = min(args.chain_steps, p["n_steps"])
    t = T.Tissue(p, device="cuda:0", trace_steps=n)
    if cfg:
        from paper_1806_10889_amd import autotune
        autotune.apply(t, cfg)
    t.restart(sim_id=4242, start_step=0)
    tm = t.step_timed(p["dt"], n)
    ce = t.trace(0, n)[0].astype(np.float64)
    basis = {"chi_events": t.stats()["chi_events"], "steps": n}
    t.close()
    busiest = float(ce.max(axis=1).mean())
    if tm["chi_launches"] != n:
        return None, basis  # several chi launches per step: no single chain per launch
    launch_ms = tm["chi_ms"] / n
    mean = float(ce.mean())
    return {"steps": n, "busiest_cell_events_per_step": busiest,
            "mean_cell_events_per_step": mean, "busiest_over_mean": busiest / max(mean, 1e-12),
            "avg_launch_ms": launch_ms,
            "ns_per_event_on_busiest_chain": launch_ms * 1e6 / max(busiest, 1.0)}, basis


def run_batched(args, torch, T, W):
    """Config-4-shaped sweep: independent tissues in one batch (one graph per
    chunk of steps).  Every member shares every launch, so each tissue's
    result is complete when the sweep is: a tissue's completion time is the
    sweep's, and its p50/p99 are taken over the repetitions."""
    probs = W.config4(n_tissues=args.batch_tissues, n_steps=args.batch_steps)
    stream = torch.cuda.current_stream()
    ts = [T.Tissue(p, device="cuda:0", stream=stream) for p in probs]
    b = T.Batch(ts, device="cuda:0", stream=stream)
    b.set_regroup(args.regroup)
    if args.refill >= 0:
        b.set_refill(args.refill)
    dt, n = probs[0]["dt"], probs[0]["n_steps"]
    basis = {"chi_events": 0, "steps": 0}

    def totals():
        chi = s_ = 0
        for t in ts:
            st = t.stats()
            chi += st["chi_events"]
            s_ += st["s_events"]
        return chi, s_

    def one(k):
        for i, t in enumerate(ts):
            t.restart(sim_id=i + 1000 * k, start_step=0)
        a = time.perf_counter()
        b.step(dt, n)
        b.sync()
        wall = time.perf_counter() - a
        chi, s_ = totals()
        basis["chi_events"] += chi
        basis["steps"] += n
        return chi, s_, wall

    # warm-up: network compilation and the graph capture of one chunk
    for i, t in enumerate(ts):
        t.restart(sim_id=i + 99000, start_step=0)
    b.step(dt, min(n, 50))
    b.sync()
    basis["chi_events"] += totals()[0]
    basis["steps"] += min(n, 50)
    tot_ev, tot_chi, tot_t, walls = 0, 0, 0.0, []
    for k in range(max(1, args.batch_reps)):
        chi, s_, wall = one(k)
        tot_ev += chi + s_
        tot_chi += chi
        tot_t += wall
        walls.append(wall)
        log(f"batched rep {k + 1}: {chi + s_} events in {wall * 1e3:.1f} ms")
    cells = sum(p["nx"] * p["ny"] for p in probs)
    out = dict(events_per_s=tot_ev / tot_t, tissues=len(probs), cells=cells, steps=n, dt=dt,
               reps=len(walls), sweep_ms_p50=pct(walls, 50) * 1e3, sweep_ms_p99=pct(walls, 99) * 1e3,
               tissue_completion_ms_p50=pct(walls, 50) * 1e3,
               tissue_completion_ms_p99=pct(walls, 99) * 1e3,
               tissue_completion="every member completes with the sweep (shared launches); "
                                 "p50/p99 over the repetitions")
    # roofline of the batched chi kernel: the same sweep once more, launched
    # eagerly with HIP events around each launch
    for i, t in enumerate(ts):
        t.restart(sim_id=i + 777, start_step=0)
    tm = b.step_timed(dt, n)
    chi_ev = totals()[0]
    basis["chi_events"] += chi_ev
    basis["steps"] += n
    ops = ops_per_chi_event_of(probs[0])
    per_launch_ms = tm["chi_ms"] / max(tm["chi_launches"], 1)
    achieved = chi_ev / max(tm["chi_launches"], 1) * ops / (per_launch_ms * 1e-3)
    kernel = chi_kernel_name(tm["chi_kernel"], bool(ts[0].stats()["jit"]), tm["chi_leaves"],
                             tm["chi_refill"])
    cnt = counter_figures("batched", [kernel], live_s_per_step=per_launch_ms * 1e-3)
    out["roofline"] = {"bound": "alu", "kernel": kernel,
                       "basis": "HIP events around every chi launch of one eager sweep",
                       "achieved": achieved / 1e12,
                       "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
                       "frac": achieved / PEAK_LANE_OPS,
                       "traffic": cnt["traffic"] if cnt else None,
                       "hbm_frac": cnt["hbm_frac"] if cnt else None, "counters": cnt,
                       "avg_launch_ms": per_launch_ms,
                       "events_per_launch": chi_ev / max(tm["chi_launches"], 1),
                       "ops_per_event": ops,
                       "s_kernel_avg_ms": tm["s_ms"] / max(tm["s_launches"], 1),
                       "timed_run": {"achieved": tot_chi * ops / tot_t / 1e12,
                                     "frac": tot_chi * ops / tot_t / PEAK_LANE_OPS,
                                     "basis": "the timed sweeps' chi events over their wall time"},
                       "counter_basis": dict(basis)}
    b.close()
    for t in ts:
        t.close()
    return out


def run_tiny(args, torch, T, W):
    """The plain tiny workload: 16 well-mixed cells on a 4x4 square lattice,
    the 4-species network, dt 0.1, T 10 (100 steps) -- a latency case: each
    simulation is 100 steps of a handful of events per cell.  By default the
    library runs such a tissue's whole call in one kernel launch; the same
    simulations step by step (one graph of 100 steps) are reported beside
    it.  Events/s and the latency per simulation and per step, the restart
    and the synchronising read of the totals included."""
    p = W.config1()
    n = p["n_steps"]

    def sims(whole):
        t = T.Tissue(p, device="cuda:0", stream=torch.cuda.current_stream())
        t.set_launch(False, 0)
        t.set_graph_chunk(n)
        t.set_whole_run(whole)
        assert t.runs_whole() == whole
        t.step(p["dt"], n)  # warm-up (the graph capture when step by step)
        t.stats()
        lat, ev = [], 0
        for k in range(args.tiny_sims):
            a = time.perf_counter()
            t.restart(sim_id=k, start_step=0)
            t.step(p["dt"], n)
            st = t.stats()
            lat.append(time.perf_counter() - a)
            ev += st["chi_events"] + st["s_events"]
        t.close()
        return {"sims": len(lat), "events_per_s": ev / sum(lat),
                "sim_latency_ms_p50": pct(lat, 50) * 1e3, "sim_latency_ms_p99": pct(lat, 99) * 1e3,
                "step_latency_us_p50": pct(lat, 50) * 1e6 / n}

    out = {"workload": "square 4x4 tissue, 16 well-mixed cells, 4 species, 7+1 reactions, "
                       "dt=0.1, T=10 (100 splitting steps)"}
    out.update(sims(True))
    out["launch"] = "the whole call in one launch of the whole-run kernel (one workgroup)"
    out["step_by_step"] = dict(sims(False), launch="one workgroup per item, one graph of 100 steps")
    return out


def run_serving(args, torch, budget_bytes=None, n_requests=None):
    """Config-5-shaped serving: Poisson arrivals replayed in real time,
    continuous batching with HBM-budgeted admission (the device's free
    memory less a margin, unless a budget is given); latency = arrival to
    result in host memory."""
    from paper_1806_10889_amd import serve
    n_req = args.serve_requests if n_requests is None else n_requests
    reqs = serve.requests_from_workload(n_req + args.serve_warmup, rate_hz=args.serve_rate)
    log(f"serving: {len(reqs)} requests generated")
    # compile the requests' network before the clock starts (the runtime
    # compiles each network structure once per process, on first use)
    from paper_1806_10889_amd import tissue as T
    T.Tissue(reqs[0].problem, device="cuda:0").close()
    be = serve.GpuBackend(lanes=args.serve_lanes, regroup=args.regroup)
    srv = serve.Server(be, max_bytes=budget_bytes, max_active=args.serve_slots,
                       quantum=args.serve_quantum, margin_bytes=args.serve_margin_gib << 30)
    st, done = srv.run(reqs, real_time=True)
    measured = [r for r in done if r.rid >= args.serve_warmup and r.status == "done"]
    lat = sorted(r.finished - r.arrival for r in measured)
    ev = sum(r.events for r in measured)
    span = max(r.finished for r in measured) - min(r.arrival for r in measured)
    out = st.summary()
    out.update({"measured_requests": len(measured), "warmup_requests": args.serve_warmup,
                "offered_rate_hz": args.serve_rate, "quantum_steps": args.serve_quantum,
                "lanes": args.serve_lanes, "batch_rebuilds": be.rebuilds,
                "budget": "device free memory less a margin" if budget_bytes is None
                          else f"{budget_bytes} bytes",
                "measured_req_per_s": len(measured) / span, "measured_events_per_s": ev / span,
                "measured_latency_ms_p50": pct(lat, 50) * 1e3,
                "measured_latency_ms_p99": pct(lat, 99) * 1e3})
    return out


# ---------------------------------------------------------------------------
# dt study: accuracy of the two splittings against the unsplit CME, and the
# time to solution of the headline tissue, as dt varies
# ---------------------------------------------------------------------------
DT_STUDY = (0.4, 0.2, 0.1, 0.05, 0.025)


def two_cell_problem(W):
    """A closed two-cell tissue (one voxel each, no diffusion) whose CME is
    solvable: cis binding/unbinding and NICD decay in each cell, the trans
    reaction over the one edge."""
    import numpy as np
    rates = np.zeros(9)
    rates[4], rates[7], rates[8] = 0.7, 0.8, 0.5
    init = np.array([[3, 1, 0, 0, 0], [1, 3, 0, 0, 0]], np.int32)
    return W.make_problem(W.model_nd5(), lattice=0, nx=2, ny=1, mesh_w=1, mesh_h=1, rates=rates,
                          trans_rate=1.5, diffusion=0.0, init_counts=init, seed=31)


def split_cme(p):
    """Reference for the accuracy study (analysis only, not a simulation
    path): the chi and S generators of the two-cell tissue on its reachable
    states, as dense matrices, and the initial distribution."""
    import numpy as np
    S = p["n_species"]
    reac = np.asarray(p["reactants"]).reshape(-1, 2)
    st = np.asarray(p["stoich"]).reshape(-1, S)

    def chi(s):
        out = []
        for cell in range(2):
            x = s[cell * S:(cell + 1) * S]
            for r in range(p["n_reactions"]):
                a, b = int(reac[r][0]), int(reac[r][1])
                c = float(p["rates"][r])
                if c == 0:
                    continue
                h = (1 if a < 0 and b < 0 else x[max(a, b)] if a < 0 or b < 0
                     else x[a] * (x[a] - 1) // 2 if a == b else x[a] * x[b])
                if h:
                    ns = list(s)
                    for q in range(S):
                        ns[cell * S + q] += int(st[r][q])
                    out.append((c * h, tuple(ns)))
        return out

    def sig(s):
        out = []
        for recv, send in ((0, 1), (1, 0)):
            h = s[recv * S + p["trans_n"]] * s[send * S + p["trans_d"]]
            if h:
                ns = list(s)
                ns[recv * S + p["trans_n"]] -= 1
                ns[send * S + p["trans_d"]] -= 1
                ns[recv * S + p["trans_i"]] += 1
                out.append((p["trans_rate"] * h, tuple(ns)))
        return out

    x0 = tuple(int(v) for v in np.asarray(p["init_counts"]).ravel())
    states, index = [x0], {x0: 0}
    q = 0
    while q < len(states):
        for _, ns in chi(states[q]) + sig(states[q]):
            if ns not in index:
                index[ns] = len(states)
                states.append(ns)
        q += 1
    n = len(states)
    Qc, Qs = np.zeros((n, n)), np.zeros((n, n))
    for Q, f in ((Qc, chi), (Qs, sig)):
        for a, s in enumerate(states):
            for rate, ns in f(s):
                Q[index[ns], a] += rate
                Q[a, a] -= rate
    p0 = np.zeros(n)
    p0[0] = 1.0
    return states, index, Qc, Qs, p0


def run_dt_study(args, torch, T, W):
    import numpy as np
    from scipy import linalg
    p2 = two_cell_problem(W)
    states, index, Qc, Qs, p0 = split_cme(p2)
    S = p2["n_species"]
    obs = np.array([s[p2["trans_i"]] for s in states], np.float64)  # I of cell 0
    T_acc = 1.2
    exact = linalg.expm((Qc + Qs) * T_acc) @ p0
    rows = []
    # GPU replicas of the two-cell tissue, one set per scheme
    R = args.dt_replicas
    reps = {}
    for scheme in ("lie", "strang"):
        ts = []
        for r in range(R):
            q = dict(p2, sim_id=r, scheme=scheme)
            ts.append(T.Tissue(q, device="cuda:0"))
        reps[scheme] = (ts, T.Batch(ts, device="cuda:0"))
    head = W.config2(n_steps=1)
    for dt in DT_STUDY:
        n = int(round(T_acc / dt))
        row = {"dt": dt}
        for scheme in ("lie", "strang"):
            Ec, Es, Eh = (linalg.expm(Qc * dt), linalg.expm(Qs * dt), linalg.expm(Qc * dt * 0.5))
            pv = p0.copy()
            for _ in range(n):
                pv = Es @ (Ec @ pv) if scheme == "lie" else Eh @ (Es @ (Eh @ pv))
            ts, b = reps[scheme]
            for r, t in enumerate(ts):
                t.restart(sim_id=r + 1000 * int(dt * 1000), start_step=0)
            b.step(dt, n)
            b.sync()
            x = np.array([t.read_counts()[p2["trans_i"]] for t in ts], np.float64)
            row[scheme] = {"law_l1": float(np.abs(pv - exact).sum()),
                           "mean_err": float(obs @ pv - obs @ exact),
                           "gpu_mean_err": float(x.mean() - obs @ exact),
                           "gpu_se": float(x.std(ddof=1) / np.sqrt(len(x)))}
        # time to solution of the headline tissue over T = args.dt_T
        n_head = int(round(args.dt_T / dt))
        for scheme in ("lie", "strang"):
            ph = dict(head, n_steps=n_head, scheme=scheme)
            t = T.Tissue(ph, device="cuda:0")
            t.set_chi_mode(2)
            t.set_launch(False, 0)
            t.set_graph_chunk(25)
            t.step(dt, n_head)  # warm-up (graph capture)
            t.restart(sim_id=5, start_step=0)
            torch.cuda.synchronize()
            a = time.perf_counter()
            t.step(dt, n_head)
            st = t.stats()
            el = time.perf_counter() - a
            row[scheme]["headline_ms"] = el * 1e3
            row[scheme]["headline_events_per_s"] = (st["chi_events"] + st["s_events"]) / el
            t.close()
        log(f"dt study: dt={dt} lie={row['lie']} strang={row['strang']}")
        rows.append(row)
    for ts, b in reps.values():
        b.close()
        for t in ts:
            t.close()
    return {"observable": "E[I] of cell 0 of a closed two-cell tissue", "T_accuracy": T_acc,
            "exact_mean": float(obs @ exact), "replicas": R,
            "headline": f"hex 64x64 tissue, 4096 cells x 4x4 voxels, T = {args.dt_T}",
            "rows": rows}


def pattern_metrics(p, counts):
    """Lateral inhibition in the paper's model: per cell, Delta and whether
    the promoter is bound; the correlation of a cell's Delta with its
    neighbours' mean (negative: neighbours inhibit each other, the
    checkerboard tendency) and the share of cells whose Delta is on the
    other side of the median from every neighbour's."""
    import numpy as np
    nx, ny = p["nx"], p["ny"]
    c = counts.reshape(nx * ny, 16, 4)
    d = c[:, :, 0].sum(axis=1).astype(np.float64).reshape(ny, nx)
    bound = float(c[:, :, 3].sum()) / (nx * ny)
    nb_sum = np.zeros_like(d)
    nb_cnt = np.zeros_like(d)
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        sh = np.roll(np.roll(d, dy, axis=0), dx, axis=1)
        valid = np.ones_like(d, bool)
        if dy == 1: valid[0, :] = False
        if dy == -1: valid[-1, :] = False
        if dx == 1: valid[:, 0] = False
        if dx == -1: valid[:, -1] = False
        nb_sum += np.where(valid, sh, 0.0)
        nb_cnt += valid
    nb_mean = nb_sum / nb_cnt
    corr = float(np.corrcoef(d.ravel(), nb_mean.ravel())[0, 1])
    med = np.median(d)
    hi = d > med
    alt = 0
    for y in range(ny):
        for x in range(nx):
            nbs = [(y + a, x + b) for a, b in ((0, 1), (0, -1), (1, 0), (-1, 0))
                   if 0 <= y + a < ny and 0 <= x + b < nx]
            alt += all(hi[q] != hi[y, x] for q in nbs)
    return {"delta_per_cell_mean": float(d.mean()), "promoter_bound_fraction": bound,
            "neighbour_correlation": corr, "checkerboard_cells": alt / (nx * ny)}


def run_notch(args, torch, T, W):
    """The paper's model (Table I as an RDME network, first-order
    signalling): the strong-scaling setup of the paper's Scaling section
    (8 x 8 cells, 10 s, dt 1.0 / 0.5 / 0.1) and a 64 x 64 tissue, time to
    solution on one GPU; then 100 s of the 64 x 64 tissue for its pattern."""
    rows = []
    for side in (8, 64):
        for dt in (1.0, 0.5, 0.1):
            n = int(round(10.0 / dt))
            p = W.config_notch(side=side, dt=dt, n_steps=n)
            t = T.Tissue(p, device="cuda:0")
            t.set_chi_mode(2)
            t.set_launch(False, 0)
            t.set_graph_chunk(min(25, n))
            t.step(dt, n)  # warm-up (graph capture)
            t.restart(sim_id=3, start_step=0)
            torch.cuda.synchronize()
            a = time.perf_counter()
            t.step(dt, n)
            st = t.stats()
            el = time.perf_counter() - a
            rows.append({"cells": side * side, "dt": dt, "steps": n, "ms": el * 1e3,
                         "events": st["chi_events"] + st["s_events"],
                         "s_events": st["s_events"],
                         "events_per_s": (st["chi_events"] + st["s_events"]) / el})
            log(f"notch: {rows[-1]}")
            t.close()
    p = W.config_notch(side=64, dt=0.1, n_steps=1000)
    t = T.Tissue(p, device="cuda:0")
    t.set_launch(False, 0)
    t.set_graph_chunk(25)
    a = time.perf_counter()
    t.step(0.1, 1000)
    st = t.stats()
    el = time.perf_counter() - a
    pat = pattern_metrics(p, t.read_counts())
    t.close()
    return {"model": "the paper's Notch model (Table I per voxel, d = 1/s), 4x4 voxels per cell, "
                     "first-order signalling at k_N", "T": 10.0, "rows": rows,
            "pattern_64x64_T100": dict(pat, ms=el * 1e3,
                                       events_per_s=(st["chi_events"] + st["s_events"]) / el)}


def run_multifidelity(args, torch, T, W):
    """Per-cell models on the paper's model: square tissues whose rim of 4
    cells keeps 4 x 4 voxels per cell while the interior cells are well
    mixed (one voxel), against the same tissue with 4 x 4 voxels everywhere.
    Time to solution over T = 10 s (dt 0.1) on 64 x 64 cells (one step's
    cost is the rim cells' event chains: latency-bound) and 256 x 256 cells
    (throughput-bound); over T = 100 s on 64 x 64, how Delta and the
    promoter state of rim and interior cells compare."""
    import numpy as np

    def per_cell(p, counts, s):
        sz = p["mesh_w"].astype(np.int64) * p["mesh_h"]
        off = np.concatenate([[0], np.cumsum(sz)[:-1]])
        return np.add.reduceat(counts.reshape(-1, 4)[:, s].astype(np.int64), off)

    rim = 4
    res = {"rows": []}
    for side in (64, 256):
        yy, xx = np.divmod(np.arange(side * side), side)
        edge = np.minimum(np.minimum(xx, side - 1 - xx), np.minimum(yy, side - 1 - yy))
        on_rim = edge < rim
        row = {"cells": side * side, "rim_cells": int(on_rim.sum())}
        for name, make in (("all_rdme", lambda n: W.config_notch(side=side, dt=0.1, n_steps=n)),
                           ("multi_fidelity", lambda n: W.config_multifidelity(
                               side=side, rim=rim, dt=0.1, n_steps=n))):
            p = make(100)
            t = T.Tissue(p, device="cuda:0")
            t.set_launch(False, 0)
            t.set_graph_chunk(25)
            t.step(0.1, 100)  # warm-up (graph capture)
            t.restart(sim_id=1, start_step=0)
            torch.cuda.synchronize()
            a = time.perf_counter()
            t.step(0.1, 100)
            st = t.stats()
            el = time.perf_counter() - a
            ev = st["chi_events"] + st["s_events"]
            r = {"voxels": int(W.n_voxels(p)), "ms_T10": el * 1e3, "events_T10": ev,
                 "events_per_s": ev / el}
            if side == 64:
                t.restart(sim_id=2, start_step=0)
                t.step(0.1, 1000)
                c = t.read_counts()
                d = per_cell(p, c, 0).astype(np.float64)
                bound = per_cell(p, c, 3)
                r.update({"rim_delta_mean_T100": float(d[on_rim].mean()),
                          "interior_delta_mean_T100": float(d[~on_rim].mean()),
                          "rim_bound_share_T100": float(bound[on_rim].mean()),
                          "interior_bound_share_T100": float(bound[~on_rim].mean())})
            t.close()
            row[name] = r
            log(f"multi-fidelity {side}x{side}: {name} {r}")
        row["speedup_T10"] = row["all_rdme"]["ms_T10"] / row["multi_fidelity"]["ms_T10"]
        res["rows"].append(row)
    res["setup"] = (f"square tissues, rim of {rim} cells at 4x4 voxels, interior cells well "
                    "mixed (1 voxel; binding constant k_a/16 per voxel; first-order signalling "
                    "at k_N*3/16 per face); dt 0.1")
    return res


def run_large_cells(args, torch, T, W):
    """Cells of 25 and 64 voxels (5x5 and 8x8 meshes) on hex tissues of
    1024, 4096 and 16384 cells, 5-species network, dt 0.05: events/s of the
    one-lane-per-cell layout (mode 0), rows of 32 or 64 lanes (mode 1), the
    compact layout with 2 or 4 lanes per cell (mode 3) and the automatic
    choice (mode 2), over 40 splitting steps replayed from graphs."""
    import numpy as np
    steps = 40
    rows = []
    for (w, h) in ((5, 5), (8, 8)):
        for side in (32, 64, 128):
            rng = np.random.Generator(np.random.PCG64(2))
            m = W.model_nd5()
            c = 10.0 ** rng.uniform(-2.0, 1.0, size=m["n_reactions"] + 1)
            x0 = rng.integers(0, 51, size=(side * side * w * h, 5)).astype(np.int32)
            p = W.make_problem(m, lattice=1, nx=side, ny=side, mesh_w=w, mesh_h=h, rates=c[:-1],
                               trans_rate=c[-1], diffusion=1.0, init_counts=x0, seed=2, dt=0.05,
                               n_steps=steps)
            row = {"cells": side * side, "mesh": f"{w}x{h}"}
            ref = None
            for mode in (0, 1, 3, 2):
                t = T.Tissue(p, device="cuda:0")
                t.set_chi_mode(mode)
                t.set_launch(False, 0)
                t.set_graph_chunk(20)
                t.step(0.05, 20)  # warm-up (graph capture)
                t.restart(sim_id=1, start_step=0)
                torch.cuda.synchronize()
                a = time.perf_counter()
                t.step(0.05, steps)
                st = t.stats()
                el = time.perf_counter() - a
                got = t.read_counts()
                if ref is None:
                    ref = got
                assert np.array_equal(got, ref), "layouts disagree"
                row[{0: "lane", 1: "rows", 3: "compact", 2: "auto"}[mode]] = \
                    (st["chi_events"] + st["s_events"]) / el
                t.close()
            log(f"large cells: {row}")
            rows.append(row)
    return {"unit": "events/s", "steps": steps, "dt": 0.05, "rows": rows}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, W, p):
    import oracle
    oracle.build(force=False)
    steps = args.cpu_steps
    a = time.perf_counter()
    r = oracle.run(p, p["dt"], steps, threads=0)
    el = time.perf_counter() - a
    cores = oracle.max_threads()
    # the same oracle on one thread, over a shorter prefix
    s1 = max(1, steps // 20)
    a = time.perf_counter()
    r1 = oracle.run(p, p["dt"], s1, threads=1)
    el1 = time.perf_counter() - a
    return {"value": (r.chi_events + r.s_events) / el, "unit": "events/s",
            "cores": cores, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"first {steps} splitting steps of the same 4096-cell tissue "
                      f"({r.chi_events + r.s_events} events, {el:.1f} s)",
            "single_thread": {"value": (r1.chi_events + r1.s_events) / el1, "unit": "events/s",
                              "sample": f"first {s1} splitting steps "
                                        f"({r1.chi_events + r1.s_events} events, {el1:.1f} s)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-steps", type=int, default=2000, help="splitting steps per simulation")
    ap.add_argument("--graph-chunk", type=int, default=50)
    ap.add_argument("--roofline-steps", type=int, default=0,
                    help="steps of the eagerly timed roofline pass (0: the whole horizon)")
    ap.add_argument("--chain-steps", type=int, default=1 << 30,
                    help="steps of the traced pass that measures the busiest cell's event chain "
                         "(at most the horizon, the default; 0: skip)")
    ap.add_argument("--dt-replicas", type=int, default=16384)
    ap.add_argument("--dt-T", type=float, default=20.0)
    ap.add_argument("--leg", choices=["all", "plain", "tiny", "uneven", "batched", "serving", "dt",
                                      "notch", "multifidelity", "large"],
                    default="all",
                    help="run one leg only (profiling runs); the JSON line then carries that leg")
    ap.add_argument("--plain-only", action="store_true", help="same as --leg plain")
    ap.add_argument("--batch-tissues", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--tiny-sims", type=int, default=50)
    ap.add_argument("--refill", type=int, default=-1,
                    help="lane refill of compact launches: idle lanes that trigger it (0 off; "
                         "-1: the library's default)")
    ap.add_argument("--regroup", type=int, default=2,
                    help="regroup cells by load before compact launches (0 off, 1 on, 2 auto)")
    ap.add_argument("--cpu-steps", type=int, default=1200)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="fixed launch shape instead of the autotuner")
    ap.add_argument("--launch", default="",
                    help="MODE,PERSISTENT,WPC,CHUNK: this launch shape instead of the autotuner")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--uneven-steps", type=int, default=1000)
    ap.add_argument("--uneven-sims", type=int, default=1)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-quantum", type=int, default=10)
    ap.add_argument("--serve-slots", type=int, default=4096)
    ap.add_argument("--serve-lanes", type=int, default=4)
    ap.add_argument("--serve-margin-gib", type=int, default=8,
                    help="serving budget: the device's free memory less this margin")
    ap.add_argument("--serve-bound-mib", type=int, default=48,
                    help="the budget of the second serving run, one that binds (0: skip it)")
    ap.add_argument("--serve-bound-requests", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the simulation "
              "path is single-GPU; sharding tissues over several GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        n = args.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "launches": 3}), flush=True)
        return
    from paper_1806_10889_amd import tissue as T
    from paper_1806_10889_amd import workloads as W

    leg = "plain" if args.plain_only else args.leg
    out = {"metric": METRIC, "unit": "events/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    if leg != "all":
        out["leg"] = leg
    if leg in ("all", "plain"):
        plain = run_single(args, torch, T, W.config2(n_steps=args.n_steps), "plain",
                           args.steps, args.warmup)
        out.update({
            "value": plain["value"], "ms_per_step": plain["elapsed"] / args.steps * 1e3,
            "config": {"workload": "hex 64x64 tissue, 4096 cells x 4x4 voxels, 5 species, "
                                   "9+1 reactions, D=1.0, dt=0.05, T=100 (2000 splitting steps)",
                       "cells": 4096, "voxels_per_cell": 16, "species": 5, "dt": 0.05,
                       "T": 0.05 * args.n_steps, "splitting_steps": args.n_steps,
                       "launch": (plain["tuned"] or {}).get(
                           "config", f"persistent, graph chunk {args.graph_chunk}"),
                       "network_kernels": "compiled per network" if plain["jit"] else "generic"},
            "plain": {"events_per_s": plain["value"], "chi_events": plain["chi"],
                      "s_events": plain["s"],
                      "sim_latency_ms_p50": pct(plain["lat"], 50) * 1e3,
                      "sim_latency_ms_p99": pct(plain["lat"], 99) * 1e3},
            "roofline": plain["roofline"],
        })
    if leg in ("all", "uneven"):
        p3 = W.config3(n_steps=args.uneven_steps)
        u = run_single(args, torch, T, p3, "uneven", args.uneven_sims, 1)
        out["uneven"] = {
            "workload": "hex 256x256 tissue, 65536 cells, V ~ lognormal(median 16, sigma 0.5) "
                        "in [4, 64], 5 species, dt=0.05, T=50 (1000 splitting steps)",
            "cells": 65536, "voxels": int(W.n_voxels(p3)), "splitting_steps": args.uneven_steps,
            "events_per_s": u["value"], "chi_events": u["chi"], "s_events": u["s"],
            "sim_latency_ms_p50": pct(u["lat"], 50) * 1e3,
            "launch": (u["tuned"] or {}).get("config"), "roofline": u["roofline"]}
    if leg in ("all", "tiny"):
        out["tiny"] = run_tiny(args, torch, T, W)
    if leg in ("all", "batched"):
        out["batched"] = run_batched(args, torch, T, W)
    if leg == "dt":
        out["dt_study"] = run_dt_study(args, torch, T, W)
    if leg == "notch":
        out["notch"] = run_notch(args, torch, T, W)
    if leg == "multifidelity":
        out["multifidelity"] = run_multifidelity(args, torch, T, W)
    if leg == "large":
        out["large_cells"] = run_large_cells(args, torch, T, W)
    if leg == "serving" or (leg == "all" and not args.no_serve):
        out["serving"] = run_serving(args, torch)
        if args.serve_bound_mib > 0:
            out["serving_bound_budget"] = run_serving(args, torch, budget_bytes=args.serve_bound_mib << 20,
                                                      n_requests=args.serve_bound_requests)
    if leg == "all" and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, W, plain["p"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
