"""Seeded synthetic inputs: reaction networks as data and the tissue workloads.

This module only draws numbers and lays out model tables; it holds none of
the simulation's arithmetic (no geometry, no propensities, no random stream
of the method).  Both the GPU path's tests and the CPU oracle take their
inputs from here.

A *problem* is a plain dict:

``lattice`` (0 square, 1 hex axial rhombus), ``nx``, ``ny``,
``mesh_w``/``mesh_h`` (per cell, 1..8), ``n_species``, ``n_reactions``,
``reactants`` [R][2] (species index or -1), ``stoich`` [R][S],
``rates`` [R] (per-voxel mass-action propensity constants),
``diffusion`` [S] (per-direction jump rate), ``trans_n``/``trans_d``/
``trans_i`` and ``trans_rate`` (the signalling reaction
N_i + D_j -> I_i; ``trans_n = -1`` disables it), ``init_counts``
[sum of voxels][S] int32 in cell order then voxel ``v = y*w + x``,
``seed`` (random-stream key), ``sim_id``, ``start_step``, ``event_cap``,
and the configured ``dt`` and ``n_steps``.

The Notch-Delta networks follow the paper's model (Results, Setup, Model:
Delta ligands and Notch receptors on the membrane, trans-activation through a
neighbour's Delta releasing NICD, NICD repressing Delta production) as
mass-action networks; the exact reaction lists are this project's reading
and are listed in the design notes.  All draws use
``numpy.random.Generator(PCG64(seed))`` in the order shapes, rates, initial
counts, arrivals.
"""
from __future__ import annotations

import math

import numpy as np

EVENT_CAP = 1 << 20

# ---------------------------------------------------------------------------
# Reaction networks (species, reactants, stoichiometry); rates drawn per config
# ---------------------------------------------------------------------------


def _net(species, reactions, trans):
    """reactions: list of (name, [reactant species...], {species: delta})."""
    S = len(species)
    idx = {s: i for i, s in enumerate(species)}
    R = len(reactions)
    reactants = np.full((max(R, 1), 2), -1, dtype=np.int32)[:R]
    stoich = np.zeros((R, S), dtype=np.int32)
    for r, (_, react, delta) in enumerate(reactions):
        for q, s in enumerate(react):
            reactants[r, q] = idx[s]
        for s, d in delta.items():
            stoich[r, idx[s]] += d
    tn, td, ti = (idx[trans[0]], idx[trans[1]], idx[trans[2]]) if trans else (-1, -1, -1)
    return dict(species=list(species), reaction_names=[x[0] for x in reactions],
                n_species=S, n_reactions=R, reactants=reactants, stoich=stoich,
                trans_n=tn, trans_d=td, trans_i=ti)


def model_nd4():
    """4 species N, D, I (NICD), R; 7 internal reactions + the S reaction."""
    return _net(
        ["N", "D", "I", "R"],
        [("prod_N", [], {"N": 1}),
         ("deg_N", ["N"], {"N": -1}),
         ("prod_D", [], {"D": 1}),
         ("deg_D", ["D"], {"D": -1}),
         ("I_to_R", ["I"], {"I": -1, "R": 1}),
         ("deg_R", ["R"], {"R": -1}),
         ("R_removes_D", ["R", "D"], {"D": -1})],
        ("N", "D", "I"))


def model_nd5():
    """ND4 plus C, the cis N.D complex: N + D -> C and C -> N + D."""
    m = _net(
        ["N", "D", "I", "R", "C"],
        [("prod_N", [], {"N": 1}),
         ("deg_N", ["N"], {"N": -1}),
         ("prod_D", [], {"D": 1}),
         ("deg_D", ["D"], {"D": -1}),
         ("I_to_R", ["I"], {"I": -1, "R": 1}),
         ("deg_R", ["R"], {"R": -1}),
         ("R_removes_D", ["R", "D"], {"D": -1}),
         ("cis_bind", ["N", "D"], {"N": -1, "D": -1, "C": 1}),
         ("cis_unbind", ["C"], {"C": -1, "N": 1, "D": 1})],
        ("N", "D", "I"))
    return m


def model_bd():
    """Birth-death: 0 -> X (k), X -> 0 (gamma X)."""
    return _net(["X"], [("birth", [], {"X": 1}), ("death", ["X"], {"X": -1})], None)


def model_diff():
    """Pure diffusion of one species."""
    return _net(["X"], [], None)


def model_tr():
    """Trans-activation only: N_i + D_j -> I_i on cell faces."""
    return _net(["N", "D", "I"], [], ("N", "D", "I"))


def model_dimer():
    """2X -> 0 (order-2 same species) and 0 -> X, for the x(x-1)/2 law."""
    return _net(["X"], [("birth", [], {"X": 1}), ("annihilate", ["X", "X"], {"X": -2})], None)


# ---------------------------------------------------------------------------
# Problem assembly
# ---------------------------------------------------------------------------


def model_notch_paper():
    """The paper's Notch model (Results, Setup, Model; Table I) as an RDME
    network: Delta (D) and NICD (I) diffuse, a promoter (G free, B bound to
    NICD) transcribes Delta while free, NICD binds and unbinds the promoter,
    D and I degrade; signalling turns a Delta in a face voxel into an NICD
    in the facing voxel of the neighbour (first order, the S operator)."""
    m = _net(
        ["D", "I", "G", "B"],
        [("transcribe", ["G"], {"D": 1}),
         ("bind", ["I", "G"], {"I": -1, "G": -1, "B": 1}),
         ("unbind", ["B"], {"B": -1, "G": 1, "I": 1}),
         ("deg_D", ["D"], {"D": -1}),
         ("deg_I", ["I"], {"I": -1})],
        None)
    m["trans_d"], m["trans_i"] = 0, 1
    m["signal"] = "first_order"
    return m


# Table I in per-voxel units for cells of 4 x 4 voxels of side h = 0.25 um:
# t_D = 1e2 /s; k_a / h^3 = 1e-18 m^3/s / (0.25 um)^3 = 64 /s; k_d = 25 /s;
# D / h^2 = 1e-12 m^2/s / (0.25 um)^2 = 16 /s per direction; k_N = 1 /s.
# The degradation rate d is not given; this project takes d = 1 /s.
NOTCH_PAPER = dict(t_D=100.0, k_a=64.0, k_d=25.0, d=1.0, D=16.0, k_N=1.0)


def config_notch(side: int = 64, dt: float = 0.1, n_steps: int = 200, seed: int = 6,
                 params: dict | None = None) -> dict:
    """The paper's tissue: identical cubic cells in a 2D square layer (at
    most four neighbours), here 4 x 4 voxels each with the promoter in voxel
    (2, 2), no Delta or NICD at the start (fluctuations break the symmetry).
    dt 0.1 s is the smallest splitting step of the paper's experiments."""
    m = model_notch_paper()
    c = dict(NOTCH_PAPER, **(params or {}))
    ncell = side * side
    x0 = np.zeros((ncell, 16, 4), dtype=np.int32)
    x0[:, 2 * 4 + 2, 2] = 1  # G = 1 in voxel (x=2, y=2)
    rates = [c["t_D"], c["k_a"], c["k_d"], c["d"], c["d"]]
    return make_problem(m, lattice=0, nx=side, ny=side, mesh_w=4, mesh_h=4, rates=rates,
                        trans_rate=c["k_N"], diffusion=[c["D"], c["D"], 0.0, 0.0],
                        init_counts=x0.reshape(-1, 4), seed=seed, dt=dt, n_steps=n_steps,
                        name=f"notch (paper's model): square {side}x{side}, 4x4 voxels")


def config_multifidelity(side: int = 64, rim: int = 4, dt: float = 0.1, n_steps: int = 200,
                         seed: int = 7, params: dict | None = None) -> dict:
    """The paper's multi-fidelity use (Discussion): detailed modules where
    cells signal, coarse ones where little happens.  Cells within `rim` of
    the tissue's border run the paper's model on 4 x 4 voxels (model 0); the
    interior cells are well mixed (one voxel of the cell's whole volume,
    16 h^3), so their NICD-promoter binding constant per voxel is k_a / 16h^3
    (model 1) and there is no intra-cell diffusion.  Signalling: a molecule
    of a 4 x 4 cell signals to a neighbour only from the 3 voxels of the
    face group towards it, 3/16 of the cell's volume, while the single voxel
    of a well-mixed cell is in every face group; so its molecules signal at
    k_N * 3/16 per face, the fine cell's per-face rate with Delta spread
    evenly (fast diffusion, D/h^2 = 16 k_N)."""
    m = model_notch_paper()
    c = dict(NOTCH_PAPER, **(params or {}))
    ncell = side * side
    yy, xx = np.divmod(np.arange(ncell), side)
    edge = np.minimum(np.minimum(xx, side - 1 - xx), np.minimum(yy, side - 1 - yy))
    fine = edge < rim
    w = np.where(fine, 4, 1).astype(np.int32)
    x0 = []
    for f in fine:
        v = np.zeros((16 if f else 1, 4), np.int32)
        v[10 if f else 0, 2] = 1  # the promoter: voxel (2, 2), or the single voxel
        x0.append(v)
    rates = [c["t_D"], c["k_a"], c["k_d"], c["d"], c["d"]]
    p = make_problem(m, lattice=0, nx=side, ny=side, mesh_w=w, mesh_h=w, rates=rates,
                     trans_rate=c["k_N"], diffusion=[c["D"], c["D"], 0.0, 0.0],
                     init_counts=np.concatenate(x0), seed=seed, dt=dt, n_steps=n_steps,
                     name=f"multi-fidelity notch: square {side}x{side}, 4x4 rim of {rim}, 1x1 inside")
    coarse = dict(reactants=m["reactants"], stoich=m["stoich"],
                  rates=[c["t_D"], c["k_a"] / 16.0, c["k_d"], c["d"], c["d"]],
                  diffusion=[0.0, 0.0, 0.0, 0.0], signal_rate=c["k_N"] * 3.0 / 16.0)
    return with_models(p, [coarse], np.where(fine, 0, 1))


def make_problem(model: dict, *, lattice: int, nx: int, ny: int, mesh_w, mesh_h,
                 rates, trans_rate: float, diffusion, init_counts, seed: int,
                 sim_id: int = 0, start_step: int = 0, dt: float = 0.1,
                 n_steps: int = 1, event_cap: int = EVENT_CAP, name: str = "") -> dict:
    n_cells = nx * ny
    mesh_w = np.broadcast_to(np.asarray(mesh_w, dtype=np.int32), (n_cells,)).copy()
    mesh_h = np.broadcast_to(np.asarray(mesh_h, dtype=np.int32), (n_cells,)).copy()
    S = model["n_species"]
    nvox = int(np.sum(mesh_w.astype(np.int64) * mesh_h))
    init_counts = np.asarray(init_counts, dtype=np.int32).reshape(nvox, S)
    return dict(
        name=name, lattice=int(lattice), nx=int(nx), ny=int(ny),
        mesh_w=mesh_w, mesh_h=mesh_h,
        n_species=S, n_reactions=model["n_reactions"],
        reactants=np.asarray(model["reactants"], dtype=np.int32).reshape(-1, 2),
        stoich=np.asarray(model["stoich"], dtype=np.int32).reshape(-1, S),
        rates=np.asarray(rates, dtype=np.float64).reshape(-1),
        diffusion=np.broadcast_to(np.asarray(diffusion, dtype=np.float64), (S,)).copy(),
        trans_n=model["trans_n"], trans_d=model["trans_d"], trans_i=model["trans_i"],
        trans_rate=float(trans_rate),
        init_counts=init_counts, seed=int(seed), sim_id=int(sim_id),
        start_step=int(start_step), event_cap=int(event_cap),
        dt=float(dt), n_steps=int(n_steps),
        species=model["species"], signal=model.get("signal", "trans"))


def with_models(problem: dict, models: list, cell_model) -> dict:
    """Per-cell networks: `models` are networks 1..K-1 over the problem's
    species (dicts with reactants, stoich, rates, diffusion and optionally
    signal_rate; model 0 is the problem's own network) and cell_model[c]
    picks each cell's.  The S reaction's species are the problem's; under
    first-order signalling a cell's molecules signal at its model's
    signal_rate (default: the problem's trans_rate)."""
    S = problem["n_species"]
    p = dict(problem)
    p["models"] = [dict(reactants=np.asarray(m["reactants"], np.int32).reshape(-1, 2),
                        stoich=np.asarray(m["stoich"], np.int32).reshape(-1, S),
                        rates=np.asarray(m["rates"], np.float64).reshape(-1),
                        diffusion=np.broadcast_to(np.asarray(m["diffusion"], np.float64), (S,)).copy(),
                        signal_rate=float(m.get("signal_rate", problem["trans_rate"])))
                   for m in models]
    p["cell_model"] = np.asarray(cell_model, dtype=np.int32).reshape(-1).copy()
    assert p["cell_model"].size == p["nx"] * p["ny"]
    assert p["cell_model"].min() >= 0 and p["cell_model"].max() <= len(models)
    return p


def n_voxels(problem: dict) -> int:
    return int(np.sum(problem["mesh_w"].astype(np.int64) * problem["mesh_h"]))


def _loguniform_rates(rng, n):
    """c = 10^U(-2, 1): log-uniform on [0.01, 10]."""
    return 10.0 ** rng.uniform(-2.0, 1.0, size=n)


def _counts(rng, nvox, S, hi=50):
    return rng.integers(0, hi + 1, size=(nvox, S), dtype=np.int64).astype(np.int32)


# ---------------------------------------------------------------------------
# The five workloads (and reduced sizes of them for tests)
# ---------------------------------------------------------------------------


def config1(seed: int = 1) -> dict:
    """4x4 square lattice, 16 well-mixed cells (1 voxel), ND4, dt=0.1, T=10."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = model_nd4()
    c = _loguniform_rates(rng, m["n_reactions"] + 1)
    x0 = _counts(rng, 16, m["n_species"])
    return make_problem(m, lattice=0, nx=4, ny=4, mesh_w=1, mesh_h=1, rates=c[:-1],
                        trans_rate=c[-1], diffusion=0.0, init_counts=x0, seed=seed,
                        dt=0.1, n_steps=100, name="config1: square 4x4, V=1, ND4")


def config2(seed: int = 2, side: int = 64, n_steps: int = 2000) -> dict:
    """Hex side x side lattice of 4x4-voxel cells, ND5, D=1.0, dt=0.05, T=100."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = model_nd5()
    c = _loguniform_rates(rng, m["n_reactions"] + 1)
    ncell = side * side
    x0 = _counts(rng, ncell * 16, m["n_species"])
    return make_problem(m, lattice=1, nx=side, ny=side, mesh_w=4, mesh_h=4, rates=c[:-1],
                        trans_rate=c[-1], diffusion=1.0, init_counts=x0, seed=seed,
                        dt=0.05, n_steps=n_steps,
                        name=f"config2: hex {side}x{side}, 4x4 voxels, ND5")


def mesh_from_voxels(V: int) -> tuple[int, int]:
    """A drawn voxel count V -> mesh (w, h): w = clamp(round(sqrt V), 2, 8),
    h = clamp(round(V / w), 2, 8)."""
    w = min(max(int(round(math.sqrt(V))), 2), 8)
    h = min(max(int(round(V / w)), 2), 8)
    return w, h


def config3(seed: int = 3, side: int = 256, n_steps: int = 1000) -> dict:
    """Hex side x side lattice with uneven cells: V ~ lognormal(median 16,
    sigma 0.5) clipped to [4, 64], ND5, dt=0.05, T=50."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = model_nd5()
    ncell = side * side
    V = np.clip(np.rint(np.exp(rng.normal(math.log(16.0), 0.5, size=ncell))), 4, 64).astype(int)
    wh = np.array([mesh_from_voxels(int(v)) for v in V], dtype=np.int32)
    c = _loguniform_rates(rng, m["n_reactions"] + 1)
    nvox = int(np.sum(wh[:, 0].astype(np.int64) * wh[:, 1]))
    x0 = _counts(rng, nvox, m["n_species"])
    return make_problem(m, lattice=1, nx=side, ny=side, mesh_w=wh[:, 0], mesh_h=wh[:, 1],
                        rates=c[:-1], trans_rate=c[-1], diffusion=1.0, init_counts=x0,
                        seed=seed, dt=0.05, n_steps=n_steps,
                        name=f"config3: hex {side}x{side}, uneven V, ND5")


def config4(seed: int = 4, n_tissues: int = 512, side_lo: int = 8, side_hi: int = 128,
            n_steps: int = 200) -> list[dict]:
    """512 independent hex tissues, sides U{8..128}, 4x4-voxel cells, ND5;
    shared base rates 10^U(-2,1) with a per-tissue, per-reaction factor
    exp(U(ln 0.5, ln 1.5)); dt=0.1, T=20.  sim_id = tissue index."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = model_nd5()
    sides = rng.integers(side_lo, side_hi + 1, size=n_tissues)
    base = _loguniform_rates(rng, m["n_reactions"] + 1)
    fac = np.exp(rng.uniform(math.log(0.5), math.log(1.5), size=(n_tissues, m["n_reactions"] + 1)))
    out = []
    for t in range(n_tissues):
        s = int(sides[t])
        c = base * fac[t]
        x0 = _counts(rng, s * s * 16, m["n_species"])
        out.append(make_problem(m, lattice=1, nx=s, ny=s, mesh_w=4, mesh_h=4, rates=c[:-1],
                                trans_rate=c[-1], diffusion=1.0, init_counts=x0, seed=seed,
                                sim_id=t, dt=0.1, n_steps=n_steps,
                                name=f"config4 tissue {t}: hex {s}x{s}"))
    return out


def config5_arrivals(seed: int = 5, n_requests: int = 2200, rate_hz: float = 200.0):
    """Poisson arrival times (seconds) of the serving stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))


def config5_request(q: int, seed: int = 5, side_lo: float = 4.0, side_hi: float = 128.0,
                    n_steps: int = 100) -> dict:
    """Request q of the serving stream: hex s x s tissue with
    s = round(exp(U(ln 4, ln 128))), per-cell (w, h) ~ U{1..4}^2, ND5, rates
    10^U(-2,1), counts U{0..50}, dt = 0.1, T = 10; sim_id = q.  Drawn from its
    own generator PCG64([seed, q]) so requests can be made lazily."""
    rng = np.random.Generator(np.random.PCG64([seed, q]))
    m = model_nd5()
    s = int(np.rint(np.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
    wh = rng.integers(1, 5, size=(s * s, 2)).astype(np.int32)
    c = _loguniform_rates(rng, m["n_reactions"] + 1)
    x0 = _counts(rng, int(np.sum(wh[:, 0].astype(np.int64) * wh[:, 1])), m["n_species"])
    return make_problem(m, lattice=1, nx=s, ny=s, mesh_w=wh[:, 0], mesh_h=wh[:, 1],
                        rates=c[:-1], trans_rate=c[-1], diffusion=1.0, init_counts=x0,
                        seed=seed, sim_id=q, dt=0.1, n_steps=n_steps,
                        name=f"request {q}: hex {s}x{s}")


# ---------------------------------------------------------------------------
# Small test problems
# ---------------------------------------------------------------------------


def birth_death(k: float, gamma: float, x0: int, *, seed: int = 11, sim_id: int = 0,
                nx: int = 1, ny: int = 1, dt: float = 0.1, n_steps: int = 10) -> dict:
    m = model_bd()
    ncell = nx * ny
    return make_problem(m, lattice=0, nx=nx, ny=ny, mesh_w=1, mesh_h=1, rates=[k, gamma],
                        trans_rate=0.0, diffusion=0.0,
                        init_counts=np.full((ncell, 1), x0, np.int32), seed=seed,
                        sim_id=sim_id, dt=dt, n_steps=n_steps, name="birth-death")


def pure_diffusion(w: int, h: int, D: float, x0_voxel: int, n0: int, *, seed: int = 12,
                   nx: int = 1, ny: int = 1, dt: float = 0.1, n_steps: int = 10) -> dict:
    m = model_diff()
    ncell = nx * ny
    x0 = np.zeros((ncell * w * h, 1), np.int32)
    for c in range(ncell):
        x0[c * w * h + x0_voxel, 0] = n0
    return make_problem(m, lattice=0, nx=nx, ny=ny, mesh_w=w, mesh_h=h, rates=[],
                        trans_rate=0.0, diffusion=D, init_counts=x0, seed=seed,
                        dt=dt, n_steps=n_steps, name="diffusion")


def random_problem(seed: int, *, lattice: int, nx: int, ny: int, model: str = "nd5",
                   mesh=None, uneven: bool = False, dt: float = 0.05, n_steps: int = 5,
                   count_hi: int = 50, sim_id: int = 0, diffusion: float = 1.0,
                   rate_lo: float = -2.0, rate_hi: float = 1.0) -> dict:
    """A random tissue for parity tests: rates 10^U(rate_lo, rate_hi), counts U{0..count_hi}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = {"nd4": model_nd4, "nd5": model_nd5, "bd": model_bd, "tr": model_tr,
         "diff": model_diff, "dimer": model_dimer}[model]()
    ncell = nx * ny
    if uneven:
        wh = rng.integers(1, 9, size=(ncell, 2)).astype(np.int32)
    else:
        w, h = mesh if mesh is not None else (4, 4)
        wh = np.tile(np.array([[w, h]], np.int32), (ncell, 1))
    c = 10.0 ** rng.uniform(rate_lo, rate_hi, size=m["n_reactions"] + 1)
    nvox = int(np.sum(wh[:, 0].astype(np.int64) * wh[:, 1]))
    x0 = _counts(rng, nvox, m["n_species"], count_hi)
    return make_problem(m, lattice=lattice, nx=nx, ny=ny, mesh_w=wh[:, 0], mesh_h=wh[:, 1],
                        rates=c[: m["n_reactions"]], trans_rate=c[-1], diffusion=diffusion,
                        init_counts=x0, seed=seed, sim_id=sim_id, dt=dt, n_steps=n_steps,
                        name=f"random {model} seed {seed}")
