"""Plain CPU FP64 oracle (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``oracle.c`` (built into ``liboracle.so`` with
gcc, no FMA contraction) through ctypes and shares no code with the GPU
library: it never imports ``paper_1806_10889_amd``.

Functions mirror the parts of the method they compute:

* :func:`philox` / :func:`uniforms` -- the counter-based stream (Philox4x32-10,
  Salmon et al. SC'11) and the two uniforms drawn per SSA event;
* :func:`plog` -- the project's natural log (atanh series, Muller's
  argument reduction);
* :func:`ring`, :func:`face_group`, :func:`voxel_neighbours`,
  :func:`lattice_edges` -- geometry (Results, Setup, Model: cubes in a 2D
  layer; coupling through a single face);
* :func:`run` -- ``n_steps`` splitting steps, chi for every cell then the
  signalling operator S over colour classes (Algorithm section: operator
  splitting; Fig. 1: chi then S every timestep); with ``problem["scheme"] ==
  "strang"`` Strang's symmetric splitting instead (chi over dt/2 with counter
  tag 0, S over dt, chi over dt/2 with tag 2).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
          "-fno-fast-math", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("mesh_w", C.POINTER(C.c_int32)), ("mesh_h", C.POINTER(C.c_int32)),
        ("n_species", C.c_int32), ("n_reactions", C.c_int32),
        ("reactants", C.POINTER(C.c_int32)), ("stoich", C.POINTER(C.c_int32)),
        ("rates", C.POINTER(C.c_double)), ("diffusion", C.POINTER(C.c_double)),
        ("trans_n", C.c_int32), ("trans_d", C.c_int32), ("trans_i", C.c_int32),
        ("signal_order", C.c_int32),
        ("trans_rate", C.c_double),
        ("seed", C.c_uint64), ("sim_id", C.c_uint32), ("start_step", C.c_uint32),
        ("event_cap", C.c_uint32), ("scheme", C.c_uint32),
        ("n_models", C.c_int32), ("pad2", C.c_int32),
        ("cell_model", C.POINTER(C.c_int32)), ("m_n_reactions", C.POINTER(C.c_int32)),
        ("m_reactants", C.POINTER(C.c_int32)), ("m_stoich", C.POINTER(C.c_int32)),
        ("m_rates", C.POINTER(C.c_double)), ("m_diffusion", C.POINTER(C.c_double)),
        ("m_signal_rate", C.POINTER(C.c_double)),
    ]


class _Stats(C.Structure):
    _fields_ = [("chi_events", C.c_uint64), ("s_events", C.c_uint64),
                ("draws", C.c_uint64), ("overflow", C.c_uint32),
                ("capped", C.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIBRARY")  # another build of oracle.c (sanitizer runs)
        if not path:
            if not os.path.exists(_LIB):
                build()
            path = _LIB
        L = C.CDLL(path)
        u32p = C.POINTER(C.c_uint32)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_uniforms.argtypes = [u32p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_plog.argtypes = [C.c_double]
        L.oracle_plog.restype = C.c_double
        i32p = C.POINTER(C.c_int32)
        ip = C.POINTER(C.c_int)
        L.oracle_ring.argtypes = [C.c_int, C.c_int, ip]
        L.oracle_face_group.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, ip]
        L.oracle_voxel_neighbours.argtypes = [C.c_int, C.c_int, C.c_int, ip]
        L.oracle_lattice_edges.argtypes = [C.c_int, C.c_int, C.c_int, i32p, i32p, i32p, i32p]
        L.oracle_lattice_neighbour.argtypes = [C.c_int] * 5
        L.oracle_num_edges.argtypes = [C.POINTER(_Problem)]
        L.oracle_run.argtypes = [C.POINTER(_Problem), C.c_double, C.c_int32, i32p,
                                 C.POINTER(_Stats), u32p, C.POINTER(C.c_uint64),
                                 u32p, C.POINTER(C.c_uint64), C.c_int32]
        L.oracle_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(ctr, key) -> tuple[int, int, int, int]:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return tuple(int(x) for x in o)


def uniforms(words) -> tuple[float, float]:
    w = np.asarray(words, dtype=np.uint32)
    u1, u2 = C.c_double(), C.c_double()
    lib().oracle_uniforms(_ptr(w, C.c_uint32), C.byref(u1), C.byref(u2))
    return u1.value, u2.value


def plog(x: float) -> float:
    return lib().oracle_plog(float(x))


def ring(w: int, h: int) -> list[int]:
    buf = (C.c_int * 64)()
    n = lib().oracle_ring(w, h, buf)
    return list(buf[:n])


def face_group(w: int, h: int, nd: int, d: int) -> list[int]:
    buf = (C.c_int * 64)()
    n = lib().oracle_face_group(w, h, nd, d, buf)
    return list(buf[:n])


def voxel_neighbours(w: int, h: int, v: int) -> list[int]:
    buf = (C.c_int * 4)()
    n = lib().oracle_voxel_neighbours(w, h, v, buf)
    return list(buf[:n])


def lattice_neighbour(lattice: int, nx: int, ny: int, cell: int, d: int) -> int:
    return lib().oracle_lattice_neighbour(lattice, nx, ny, cell, d)


def lattice_edges(lattice: int, nx: int, ny: int):
    """(i, j, d, colour) arrays, ranked by (colour, i)."""
    E = lib().oracle_lattice_edges(lattice, nx, ny, None, None, None, None)
    arrs = [np.zeros(max(E, 1), dtype=np.int32) for _ in range(4)]
    lib().oracle_lattice_edges(lattice, nx, ny, *[_ptr(a, C.c_int32) for a in arrs])
    return tuple(a[:E] for a in arrs)


@dataclass
class RunResult:
    counts: np.ndarray
    chi_events: int
    s_events: int
    draws: int
    overflow: bool
    capped: bool
    chi_trace_events: np.ndarray | None = None
    chi_trace_t: np.ndarray | None = None
    s_trace_events: np.ndarray | None = None
    s_trace_t: np.ndarray | None = None


def run(problem: dict, dt: float, n_steps: int, counts=None, start_step=None,
        trace: bool = False, threads: int = 0) -> RunResult:
    """Advance ``problem`` (a dict as produced by the workload generator) by
    ``n_steps`` splitting steps of length ``dt``.  ``counts`` defaults to the
    problem's initial counts; the input array is not modified."""
    p = problem
    cnt = np.array(p["init_counts"] if counts is None else counts, dtype=np.int32, copy=True).ravel()
    mesh_w = np.ascontiguousarray(p["mesh_w"], dtype=np.int32)
    mesh_h = np.ascontiguousarray(p["mesh_h"], dtype=np.int32)
    reactants = np.ascontiguousarray(p["reactants"], dtype=np.int32).reshape(-1)
    stoich = np.ascontiguousarray(p["stoich"], dtype=np.int32).reshape(-1)
    rates = np.ascontiguousarray(p["rates"], dtype=np.float64)
    diffusion = np.ascontiguousarray(p["diffusion"], dtype=np.float64)
    if reactants.size == 0:
        reactants = np.zeros(2, dtype=np.int32)
        stoich = np.zeros(1, dtype=np.int32)
        rates = np.zeros(1, dtype=np.float64)
    pr = _Problem()
    pr.lattice = int(p["lattice"]); pr.nx = int(p["nx"]); pr.ny = int(p["ny"])
    pr.mesh_w = _ptr(mesh_w, C.c_int32); pr.mesh_h = _ptr(mesh_h, C.c_int32)
    pr.n_species = int(p["n_species"]); pr.n_reactions = int(p["n_reactions"])
    pr.reactants = _ptr(reactants, C.c_int32); pr.stoich = _ptr(stoich, C.c_int32)
    pr.rates = _ptr(rates, C.c_double); pr.diffusion = _ptr(diffusion, C.c_double)
    pr.trans_n = int(p["trans_n"]); pr.trans_d = int(p["trans_d"]); pr.trans_i = int(p["trans_i"])
    pr.trans_rate = float(p["trans_rate"])
    pr.seed = int(p["seed"]); pr.sim_id = int(p["sim_id"])
    pr.start_step = int(p.get("start_step", 0) if start_step is None else start_step)
    pr.event_cap = int(p.get("event_cap", 1 << 20))
    pr.scheme = 1 if p.get("scheme", "lie") == "strang" else 0
    pr.signal_order = 1 if p.get("signal", "trans") == "first_order" else 2
    ncell = pr.nx * pr.ny
    keep = []
    if p.get("models"):
        # model 0 = the problem's own network, then problem["models"]; tables
        # padded to 16 reactions
        S = pr.n_species
        allm = [dict(reactants=p["reactants"], stoich=p["stoich"], rates=p["rates"],
                     diffusion=p["diffusion"])] + list(p["models"])
        K = len(allm)
        nr = np.zeros(K, np.int32)
        mre = np.full((K, 16, 2), -1, np.int32)
        mst = np.zeros((K, 16, S), np.int32)
        mra = np.zeros((K, 16), np.float64)
        mdi = np.zeros((K, S), np.float64)
        msr = np.array([float(p["trans_rate"])] +
                       [float(md.get("signal_rate", p["trans_rate"])) for md in p["models"]])
        for m, md in enumerate(allm):
            r = np.asarray(md["reactants"], np.int32).reshape(-1, 2)
            nr[m] = r.shape[0]
            mre[m, :nr[m]] = r
            mst[m, :nr[m]] = np.asarray(md["stoich"], np.int32).reshape(-1, S)
            mra[m, :nr[m]] = np.asarray(md["rates"], np.float64)
            mdi[m] = np.asarray(md["diffusion"], np.float64)
        cm = np.ascontiguousarray(p["cell_model"], dtype=np.int32)
        keep = [nr, mre, mst, mra, mdi, msr, cm]
        pr.n_models = K
        pr.cell_model = _ptr(cm, C.c_int32)
        pr.m_n_reactions = _ptr(nr, C.c_int32)
        pr.m_reactants = _ptr(mre, C.c_int32)
        pr.m_stoich = _ptr(mst, C.c_int32)
        pr.m_rates = _ptr(mra, C.c_double)
        pr.m_diffusion = _ptr(mdi, C.c_double)
        pr.m_signal_rate = _ptr(msr, C.c_double)
    else:
        pr.n_models = 1
    E = lib().oracle_num_edges(C.byref(pr))
    st = _Stats()
    tr = [None] * 4
    if trace:
        tr = [np.zeros(max(n_steps * ncell, 1), np.uint32), np.zeros(max(n_steps * ncell, 1), np.uint64),
              np.zeros(max(n_steps * E, 1), np.uint32), np.zeros(max(n_steps * E, 1), np.uint64)]
    ptrs = [None if a is None else _ptr(a, ct) for a, ct in
            zip(tr, [C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint64])]
    lib().oracle_run(C.byref(pr), float(dt), int(n_steps), _ptr(cnt, C.c_int32), C.byref(st),
                     *ptrs, int(threads))
    res = RunResult(cnt, st.chi_events, st.s_events, st.draws, bool(st.overflow), bool(st.capped))
    if trace:
        res.chi_trace_events = tr[0][: n_steps * ncell].reshape(n_steps, ncell)
        res.chi_trace_t = tr[1][: n_steps * ncell].reshape(n_steps, ncell)
        res.s_trace_events = tr[2][: n_steps * E].reshape(n_steps, E)
        res.s_trace_t = tr[3][: n_steps * E].reshape(n_steps, E)
    return res


def max_threads() -> int:
    return lib().oracle_max_threads()
