"""Autotuner of the launch shape.

The launch shape -- chi kernel (one lane per cell with a full sum tree, the
compact layout with one lane per 16 voxels of a cell, or one row of lanes
per cell), persistent work queue or one workgroup per item, resident workgroups
per CU, steps per captured HIP graph -- never changes results (every choice
is bit-identical), only speed.  `tune` times candidate shapes on the
workload -- a single tissue on the tissue itself, a batch on clones of its
problems -- restarted before each candidate so that all see the same work,
keeps the fastest, caches it on disk under a signature of the workload's
shape and applies it.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

CACHE = os.environ.get("TISSUE_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "tissue_autotune.json"))


def signature(problems) -> str:
    """Shape of a workload: per problem the lattice, size, mesh histogram and
    network structure (not the rates, counts or seeds)."""
    h = hashlib.sha1()
    for p in problems:
        V = (np.asarray(p["mesh_w"], np.int64) * np.asarray(p["mesh_h"], np.int64))
        hist = np.bincount(V, minlength=65)
        h.update(repr((p["lattice"], p["nx"], p["ny"], p["n_species"], p["n_reactions"],
                       np.asarray(p["reactants"]).tolist(), np.asarray(p["stoich"]).tolist(),
                       (np.asarray(p["diffusion"]) > 0).tolist(), p["trans_n"] >= 0,
                       hist.tolist())).encode())
    return h.hexdigest()


def candidates(max_voxels: int, cells: int = 0):
    out = []
    # every mode covers every leaf-count class (the compact layout with 1, 2
    # or 4 lanes per cell; rows of 16, 32 or 64 lanes); auto mixes them per
    # class; listed so that the likelier winners come first.  With 64 Ki
    # cells or more every SIMD holds 64 compact lanes of work: one row of
    # lanes per cell (modes 1, 4) or the full-LDS lane layout (mode 0) only
    # cost more issue slots per event there, and are not timed
    if cells >= 65536:
        modes = [2, 3]
    else:
        modes = [0, 1, 4, 3, 2] if max_voxels <= 16 else [2, 3, 1, 0, 4]
    for mode in modes:
        for persistent, wpc in [(1, 0), (0, 0), (1, 2), (1, 8)]:
            for chunk in (25, 100):
                out.append(dict(chi_mode=mode, persistent=persistent, wpc=wpc, graph_chunk=chunk))
    return out


def apply(target, cfg: dict):
    target.set_chi_mode(cfg["chi_mode"])
    target.set_launch(bool(cfg["persistent"]), cfg["wpc"])
    target.set_graph_chunk(cfg["graph_chunk"])


def _load_cache():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def tune(problems, dt: float, steps: int = 50, reps: int = 2, device="cuda:0", target=None,
         use_cache: bool = True, log=None) -> dict:
    """Pick the fastest launch shape for `problems` (one tissue, or a batch
    when several) and apply it to `target` (a Tissue or Batch) if given.
    A single tissue is timed on `target` itself (restarted before every
    candidate and at the end), which spares a second copy of its state and
    its streams; a batch is timed on clones."""
    from . import tissue as T
    sig = signature(problems)
    cache = _load_cache() if use_cache else {}
    if sig in cache:
        best = cache[sig]["config"]
        if target is not None:
            apply(target, best)
        return dict(cache[sig], cached=True)
    own = not (len(problems) == 1 and isinstance(target, T.Tissue))
    clones = [T.Tissue(p, device=device) for p in problems] if own else [target]
    runner = clones[0] if len(clones) == 1 else T.Batch(clones, device=device)
    vmax = max(int(np.max(np.asarray(p["mesh_w"]) * np.asarray(p["mesh_h"]))) for p in problems)
    ncells = sum(int(p["nx"]) * int(p["ny"]) for p in problems)
    results = []
    for cfg in candidates(vmax, ncells):
        apply(runner, cfg)
        # at least one whole graph chunk, so that a candidate's steps run
        # from its graph and not eagerly
        n = max(steps, cfg["graph_chunk"])
        times = []
        for _ in range(reps + 1):  # the first run captures the graph
            for t in clones:
                t.restart(t.problem["sim_id"], 0)
            a = time.perf_counter()
            runner.step(dt, n)
            runner.sync()
            times.append(time.perf_counter() - a)
        ms_per_step = 1e3 * min(times[1:]) / n
        results.append((ms_per_step, cfg))
        if log:
            log(f"autotune {cfg}: {ms_per_step * n:.2f} ms / {n} steps")
    results.sort(key=lambda x: x[0])
    best = results[0][1]
    entry = {"config": best, "ms_per_step": results[0][0],
             "worst_ms_per_step": results[-1][0], "candidates": len(results)}
    cache[sig] = entry
    if use_cache:
        _save_cache(cache)
    if target is not None:
        apply(target, best)
    if not own:
        target.restart(target.problem["sim_id"], int(target.problem.get("start_step", 0)))
        return dict(entry, cached=False)
    if runner is not clones[0]:
        runner.close()
    for t in clones:
        t.close()
    return dict(entry, cached=False)
