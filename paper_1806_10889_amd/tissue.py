"""ctypes binding of libtissue.so (include/tissue.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of the library.  PyTorch provides the device memory (a uint8 tensor
per tissue or batch) and, optionally, the stream.  Importing this module
loads the library and raises if it has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: its bundled HIP runtime and the system one share a soname, so
# whichever is loaded first serves the whole process; libtissue must bind to
# the runtime that owns torch's device memory and streams.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# TISSUE_LIBRARY may name another build of the same library (same ABI)
LIB_PATH = os.environ.get("TISSUE_LIBRARY") or os.path.join(_HERE, "libtissue.so")

OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, EBUSY, ESTATE, ELIMIT = 0, -1, -2, -3, -4, -5, -6, -7
FLAG_TRACE = 1
FLAG_NO_JIT = 2
FLAG_STRANG = 4
FLAG_SIGNAL_FIRST_ORDER = 8
STATS_BLOCK_BYTES = 64
ABI_VERSION = 2


class TissueError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Desc(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("lattice", C.c_uint32),
        ("nx", C.c_uint32), ("ny", C.c_uint32),
        ("mesh_w", C.POINTER(C.c_uint8)), ("mesh_h", C.POINTER(C.c_uint8)),
        ("mesh_w0", C.c_uint32), ("mesh_h0", C.c_uint32),
        ("n_species", C.c_uint32), ("n_reactions", C.c_uint32),
        ("reactants", C.POINTER(C.c_int32)), ("stoich", C.POINTER(C.c_int32)),
        ("rates", C.POINTER(C.c_double)), ("diffusion", C.POINTER(C.c_double)),
        ("trans_n", C.c_int32), ("trans_d", C.c_int32), ("trans_i", C.c_int32),
        ("flags", C.c_uint32), ("trans_rate", C.c_double),
        ("init_counts", C.POINTER(C.c_int32)),
        ("seed", C.c_uint64), ("sim_id", C.c_uint32), ("start_step", C.c_uint32),
        ("event_cap", C.c_uint32), ("trace_steps", C.c_uint32),
        ("n_models", C.c_uint32), ("models", C.c_void_p), ("cell_model", C.POINTER(C.c_uint8)),
    ]


class Model(C.Structure):
    """One more intracellular network (per-cell models)."""
    _fields_ = [
        ("n_reactions", C.c_uint32),
        ("reactants", C.POINTER(C.c_int32)), ("stoich", C.POINTER(C.c_int32)),
        ("rates", C.POINTER(C.c_double)), ("diffusion", C.POINTER(C.c_double)),
        ("signal_rate", C.c_double),
    ]


class Stats(C.Structure):
    _fields_ = [("chi_events", C.c_uint64), ("s_events", C.c_uint64), ("draws", C.c_uint64),
                ("steps_done", C.c_uint32), ("overflow", C.c_uint32), ("capped", C.c_uint32),
                ("n_cells", C.c_uint32), ("n_edges", C.c_uint32), ("n_voxels", C.c_uint32),
                ("jit", C.c_uint32)]


class Timing(C.Structure):
    _fields_ = [("chi_ms", C.c_double), ("s_ms", C.c_double), ("total_ms", C.c_double),
                ("chi_launches", C.c_uint32), ("s_launches", C.c_uint32),
                ("chi_kernel", C.c_int32), ("chi_leaves", C.c_int32), ("chi_refill", C.c_int32)]


EXPORTS = [
    "tissue_required_bytes", "tissue_create", "tissue_step", "tissue_read_counts",
    "tissue_read_stats", "tissue_read_trace", "tissue_restart", "tissue_write_counts",
    "tissue_set_launch", "tissue_set_chi_mode", "tissue_set_graph_chunk", "tissue_step_timed",
    "tissue_stats_enqueue", "tissue_stats_decode",
    "tissue_destroy", "tissue_batch_set_chi_mode", "tissue_network_check",
    "tissue_batch_set_graph_chunk", "tissue_set_regroup", "tissue_batch_set_regroup",
    "tissue_batch_required_bytes", "tissue_batch_create", "tissue_batch_step",
    "tissue_batch_step_timed", "tissue_batch_set_launch", "tissue_batch_sync",
    "tissue_batch_destroy", "tissue_strerror", "tissue_last_error", "tissue_device_cus",
    "tissue_batch_step_static", "tissue_set_refill", "tissue_batch_set_refill",
    "tissue_batch_set_members", "tissue_set_whole_run", "tissue_batch_set_whole_run",
    "tissue_runs_whole", "tissue_batch_runs_whole",
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1806_10889_amd/build.py "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, u32, sz, dbl = C.c_void_p, C.c_int32, C.c_uint32, C.c_size_t, C.c_double
    pD = C.POINTER(Desc)
    sig = {
        "tissue_required_bytes": (sz, [pD]),
        "tissue_network_check": (C.c_int, [pD]),
        "tissue_create": (C.c_int, [pD, vp, sz, vp, C.POINTER(vp)]),
        "tissue_step": (C.c_int, [vp, dbl, i32]),
        "tissue_read_counts": (C.c_int, [vp, C.POINTER(C.c_int32), sz]),
        "tissue_read_stats": (C.c_int, [vp, C.POINTER(Stats)]),
        "tissue_read_trace": (C.c_int, [vp, u32, u32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)]),
        "tissue_restart": (C.c_int, [vp, u32, u32]),
        "tissue_write_counts": (C.c_int, [vp, C.POINTER(C.c_int32), sz]),
        "tissue_set_launch": (C.c_int, [vp, i32, i32]),
        "tissue_set_graph_chunk": (C.c_int, [vp, i32]),
        "tissue_set_regroup": (C.c_int, [vp, i32]),
        "tissue_batch_set_regroup": (C.c_int, [vp, i32]),
        "tissue_set_chi_mode": (C.c_int, [vp, i32]),
        "tissue_batch_set_chi_mode": (C.c_int, [vp, i32]),
        "tissue_batch_set_graph_chunk": (C.c_int, [vp, i32]),
        "tissue_step_timed": (C.c_int, [vp, dbl, i32, C.POINTER(Timing)]),
        "tissue_stats_enqueue": (C.c_int, [vp, vp]),
        "tissue_stats_decode": (C.c_int, [vp, vp, C.POINTER(Stats)]),
        "tissue_destroy": (C.c_int, [vp]),
        "tissue_batch_required_bytes": (sz, [C.POINTER(vp), i32]),
        "tissue_batch_create": (C.c_int, [C.POINTER(vp), i32, vp, sz, vp, C.POINTER(vp)]),
        "tissue_batch_step": (C.c_int, [vp, dbl, i32]),
        "tissue_batch_step_timed": (C.c_int, [vp, dbl, i32, C.POINTER(Timing)]),
        "tissue_batch_set_launch": (C.c_int, [vp, i32, i32]),
        "tissue_batch_sync": (C.c_int, [vp]),
        "tissue_batch_destroy": (C.c_int, [vp]),
        "tissue_strerror": (C.c_char_p, [C.c_int]),
        "tissue_last_error": (C.c_char_p, []),
        "tissue_device_cus": (C.c_int, [C.POINTER(C.c_int32)]),
        "tissue_batch_step_static": (C.c_int, [C.POINTER(vp), i32, dbl, i32, vp]),
        "tissue_set_refill": (C.c_int, [vp, i32]),
        "tissue_batch_set_refill": (C.c_int, [vp, i32]),
        "tissue_set_whole_run": (C.c_int, [vp, i32]),
        "tissue_batch_set_whole_run": (C.c_int, [vp, i32]),
        "tissue_runs_whole": (C.c_int, [vp]),
        "tissue_batch_runs_whole": (C.c_int, [vp]),
        "tissue_batch_set_members": (C.c_int, [vp, C.POINTER(vp), i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def _check(rc: int, what: str, allow=()):
    if rc != OK and rc not in allow:
        detail = lib.tissue_last_error().decode()
        raise TissueError(rc, f"{what}: {lib.tissue_strerror(rc).decode()}: {detail}")
    return rc


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _stream_handle(stream):
    if stream is None:
        return None
    return C.c_void_p(int(stream.cuda_stream))


class _DescHolder:
    """A filled Desc plus the numpy arrays its pointers refer to."""

    def __init__(self, problem: dict, trace_steps: int = 0, jit: bool = True):
        p = problem
        self.mesh_w = np.ascontiguousarray(p["mesh_w"], dtype=np.uint8)
        self.mesh_h = np.ascontiguousarray(p["mesh_h"], dtype=np.uint8)
        self.reactants = np.ascontiguousarray(np.asarray(p["reactants"], np.int32).reshape(-1))
        self.stoich = np.ascontiguousarray(np.asarray(p["stoich"], np.int32).reshape(-1))
        self.rates = np.ascontiguousarray(p["rates"], dtype=np.float64)
        self.diffusion = np.ascontiguousarray(p["diffusion"], dtype=np.float64)
        self.counts = np.ascontiguousarray(np.asarray(p["init_counts"], np.int32).reshape(-1))
        d = Desc()
        d.abi_version = ABI_VERSION
        d.lattice = int(p["lattice"])
        d.nx, d.ny = int(p["nx"]), int(p["ny"])
        d.mesh_w, d.mesh_h = _p(self.mesh_w, C.c_uint8), _p(self.mesh_h, C.c_uint8)
        d.n_species, d.n_reactions = int(p["n_species"]), int(p["n_reactions"])
        d.reactants, d.stoich = _p(self.reactants, C.c_int32), _p(self.stoich, C.c_int32)
        d.rates, d.diffusion = _p(self.rates, C.c_double), _p(self.diffusion, C.c_double)
        d.trans_n, d.trans_d, d.trans_i = int(p["trans_n"]), int(p["trans_d"]), int(p["trans_i"])
        d.trans_rate = float(p["trans_rate"])
        d.init_counts = _p(self.counts, C.c_int32)
        d.seed = int(p["seed"])
        d.sim_id = int(p["sim_id"])
        d.start_step = int(p.get("start_step", 0))
        d.event_cap = int(p.get("event_cap", 0))
        scheme = p.get("scheme", "lie")
        if scheme not in ("lie", "strang"):
            raise ValueError(f"scheme must be 'lie' or 'strang', not {scheme!r}")
        signal = p.get("signal", "trans")
        if signal not in ("trans", "first_order"):
            raise ValueError(f"signal must be 'trans' or 'first_order', not {signal!r}")
        d.flags = ((FLAG_TRACE if trace_steps > 0 else 0) | (0 if jit else FLAG_NO_JIT) |
                   (FLAG_STRANG if scheme == "strang" else 0) |
                   (FLAG_SIGNAL_FIRST_ORDER if signal == "first_order" else 0))
        d.trace_steps = int(trace_steps)
        models = p.get("models") or []
        if models:
            # networks 1..K-1 over the problem's species; cell_model picks each cell's
            self.m_tables = []
            self.m_structs = (Model * len(models))()
            for m, md in enumerate(models):
                t = [np.ascontiguousarray(np.asarray(md["reactants"], np.int32).reshape(-1)),
                     np.ascontiguousarray(np.asarray(md["stoich"], np.int32).reshape(-1)),
                     np.ascontiguousarray(md["rates"], dtype=np.float64).reshape(-1),
                     np.ascontiguousarray(md["diffusion"], dtype=np.float64).reshape(-1)]
                self.m_tables.append(t)
                ms = self.m_structs[m]
                ms.n_reactions = int(t[2].size)
                ms.reactants, ms.stoich = _p(t[0], C.c_int32), _p(t[1], C.c_int32)
                ms.rates, ms.diffusion = _p(t[2], C.c_double), _p(t[3], C.c_double)
                ms.signal_rate = float(md.get("signal_rate", p["trans_rate"]))
            cm = np.asarray(p["cell_model"]).reshape(-1)
            if cm.size != d.nx * d.ny or cm.min() < 0 or cm.max() > 255:
                raise ValueError("cell_model must give each cell a network index in 0..255")
            self.cell_model = np.ascontiguousarray(cm, dtype=np.uint8)
            d.n_models = len(models)
            d.models = C.cast(self.m_structs, C.c_void_p)
            d.cell_model = _p(self.cell_model, C.c_uint8)
        self.desc = d


def required_bytes(problem: dict, trace_steps: int = 0) -> int:
    h = _DescHolder(problem, trace_steps)
    return int(lib.tissue_required_bytes(C.byref(h.desc)))


def network_check(problem: dict) -> None:
    """Compile the chi kernels for the problem's network (no device needed)."""
    h = _DescHolder(problem)
    _check(lib.tissue_network_check(C.byref(h.desc)), "tissue_network_check")


def device_cus() -> int:
    n = C.c_int32()
    _check(lib.tissue_device_cus(C.byref(n)), "tissue_device_cus")
    return n.value


class Tissue:
    """One tissue resident in a torch-allocated device buffer."""

    def __init__(self, problem: dict, device="cuda:0", stream=None, trace_steps: int = 0,
                 buffer=None, jit: bool = True):
        import torch
        self.problem = problem
        self._h = _DescHolder(problem, trace_steps, jit)
        need = int(lib.tissue_required_bytes(C.byref(self._h.desc)))
        if need == 0:  # invalid descriptor: tissue_create reports why, before any device work
            _check(lib.tissue_create(C.byref(self._h.desc), None, 0, None, C.byref(C.c_void_p())),
                   "tissue_create")
        self.bytes = need
        if buffer is None:
            buffer = torch.empty(need + 256, dtype=torch.uint8, device=device)
        self.buffer = buffer  # keeps the device memory alive
        addr = buffer.data_ptr()
        aligned = (addr + 255) // 256 * 256
        avail = buffer.numel() - (aligned - addr)
        self.stream = stream
        h = C.c_void_p()
        _check(lib.tissue_create(C.byref(self._h.desc), C.c_void_p(aligned), avail,
                                 _stream_handle(stream), C.byref(h)), "tissue_create")
        self.handle = h
        self.n_values = int(self._h.counts.size)

    def step(self, dt: float, n_steps: int):
        _check(lib.tissue_step(self.handle, float(dt), int(n_steps)), "tissue_step")

    def step_timed(self, dt: float, n_steps: int) -> dict:
        t = Timing()
        _check(lib.tissue_step_timed(self.handle, float(dt), int(n_steps), C.byref(t)), "tissue_step_timed")
        return dict(chi_ms=t.chi_ms, s_ms=t.s_ms, total_ms=t.total_ms,
                    chi_launches=t.chi_launches, s_launches=t.s_launches,
                    chi_kernel=t.chi_kernel, chi_leaves=t.chi_leaves, chi_refill=t.chi_refill)

    def read_counts(self, allow_flags: bool = False) -> np.ndarray:
        out = np.empty(self.n_values, dtype=np.int32)
        allow = (EOVERFLOW, ELIMIT) if allow_flags else ()
        _check(lib.tissue_read_counts(self.handle, _p(out, C.c_int32), out.size), "tissue_read_counts", allow)
        return out

    def stats(self) -> dict:
        s = Stats()
        _check(lib.tissue_read_stats(self.handle, C.byref(s)), "tissue_read_stats")
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def stats_enqueue(self, dst_ptr: int):
        """Enqueue a copy of the statistics block (STATS_BLOCK_BYTES) to host
        address dst_ptr (pinned) on the tissue's stream; decode it with
        stats_decode once the stream has passed that point."""
        _check(lib.tissue_stats_enqueue(self.handle, C.c_void_p(int(dst_ptr))), "tissue_stats_enqueue")

    def stats_decode(self, src_ptr: int) -> dict:
        s = Stats()
        _check(lib.tissue_stats_decode(self.handle, C.c_void_p(int(src_ptr)), C.byref(s)),
               "tissue_stats_decode")
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def trace(self, first_step: int, n_steps: int):
        st = self.stats()
        nc, ne = st["n_cells"], st["n_edges"]
        ce = np.zeros(max(n_steps * nc, 1), np.uint32)
        ct = np.zeros(max(n_steps * nc, 1), np.uint64)
        se = np.zeros(max(n_steps * ne, 1), np.uint32)
        stt = np.zeros(max(n_steps * ne, 1), np.uint64)
        _check(lib.tissue_read_trace(self.handle, int(first_step), int(n_steps), _p(ce, C.c_uint32),
                                     _p(ct, C.c_uint64), _p(se, C.c_uint32), _p(stt, C.c_uint64)),
               "tissue_read_trace")
        return (ce[: n_steps * nc].reshape(n_steps, nc), ct[: n_steps * nc].reshape(n_steps, nc),
                se[: n_steps * ne].reshape(n_steps, ne), stt[: n_steps * ne].reshape(n_steps, ne))

    def restart(self, sim_id: int, start_step: int = 0):
        _check(lib.tissue_restart(self.handle, int(sim_id), int(start_step)), "tissue_restart")

    def write_counts(self, counts):
        a = np.ascontiguousarray(np.asarray(counts, np.int32).reshape(-1))
        _check(lib.tissue_write_counts(self.handle, _p(a, C.c_int32), a.size), "tissue_write_counts")

    def set_launch(self, persistent: bool, workgroups_per_cu: int = 0):
        _check(lib.tissue_set_launch(self.handle, int(bool(persistent)), int(workgroups_per_cu)),
               "tissue_set_launch")

    def set_chi_mode(self, mode: int):
        """0 = one lane per cell, 1 = one 16-lane row per cell (<= 16 voxels), 2 = auto."""
        _check(lib.tissue_set_chi_mode(self.handle, int(mode)), "tissue_set_chi_mode")

    def set_graph_chunk(self, steps: int):
        _check(lib.tissue_set_graph_chunk(self.handle, int(steps)), "tissue_set_graph_chunk")

    def set_refill(self, min_idle_lanes: int):
        """Lane refill of compact launches (0 off, 1..64 idle lanes; results unchanged)."""
        _check(lib.tissue_set_refill(self.handle, int(min_idle_lanes)), "tissue_set_refill")

    def set_whole_run(self, enable: bool):
        """Small tissues: every step of a call in one kernel launch (the
        default; results unchanged)."""
        _check(lib.tissue_set_whole_run(self.handle, int(bool(enable))), "tissue_set_whole_run")

    def runs_whole(self) -> bool:
        """Whether step() runs this tissue in the whole-run kernel."""
        rc = lib.tissue_runs_whole(self.handle)
        _check(min(rc, 0), "tissue_runs_whole")
        return rc == 1

    def set_regroup(self, mode: int):
        """0 off, 1 on, 2 automatic: the load-ordered regroup pass before
        compact-layout chi launches (results are unchanged)."""
        _check(lib.tissue_set_regroup(self.handle, int(mode)), "tissue_set_regroup")

    def sync(self):
        self.stats()

    def close(self):
        """Destroy the handle (TISSUE_ESTATE while a live batch holds it)."""
        if getattr(self, "handle", None):
            _check(lib.tissue_destroy(self.handle), "tissue_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STATIC_WORKSPACE_BYTES = 32 << 20  # TISSUE_STATIC_WORKSPACE_BYTES


def batch_step_static(tissues, dt: float, n_steps: int, stream=None):
    """tissue_batch_step_static: the tissues advanced together with the
    batch's work lists in the library's static device workspace (no batch
    handle, no allocation)."""
    arr = (C.c_void_p * len(tissues))(*[t.handle.value for t in tissues])
    _check(lib.tissue_batch_step_static(arr, len(tissues), float(dt), int(n_steps),
                                        _stream_handle(stream)), "tissue_batch_step_static")


class Batch:
    """Many tissues advanced by shared launches (one HIP graph per chunk of steps).
    capacity_bytes: a larger work-list buffer than these members need, room
    for set_members to admit more later."""

    def __init__(self, tissues, device="cuda:0", stream=None, capacity_bytes: int = 0):
        import torch
        self.tissues = list(tissues)
        arr = (C.c_void_p * len(self.tissues))(*[t.handle.value for t in self.tissues])
        self._arr = arr
        need = int(lib.tissue_batch_required_bytes(arr, len(self.tissues)))
        if need == 0:
            _check(lib.tissue_batch_create(arr, len(self.tissues), None, 0, None, C.byref(C.c_void_p())),
                   "tissue_batch_create")
        need = max(need, int(capacity_bytes))
        self.buffer = torch.empty(need + 256, dtype=torch.uint8, device=device)
        addr = self.buffer.data_ptr()
        aligned = (addr + 255) // 256 * 256
        h = C.c_void_p()
        _check(lib.tissue_batch_create(arr, len(self.tissues), C.c_void_p(aligned),
                                       self.buffer.numel() - (aligned - addr),
                                       _stream_handle(stream), C.byref(h)), "tissue_batch_create")
        self.handle = h

    def step(self, dt: float, n_steps: int):
        _check(lib.tissue_batch_step(self.handle, float(dt), int(n_steps)), "tissue_batch_step")

    def step_timed(self, dt: float, n_steps: int) -> dict:
        t = Timing()
        _check(lib.tissue_batch_step_timed(self.handle, float(dt), int(n_steps), C.byref(t)),
               "tissue_batch_step_timed")
        return dict(chi_ms=t.chi_ms, s_ms=t.s_ms, total_ms=t.total_ms,
                    chi_launches=t.chi_launches, s_launches=t.s_launches,
                    chi_kernel=t.chi_kernel, chi_leaves=t.chi_leaves, chi_refill=t.chi_refill)

    def set_launch(self, persistent: bool, workgroups_per_cu: int = 0):
        _check(lib.tissue_batch_set_launch(self.handle, int(bool(persistent)), int(workgroups_per_cu)),
               "tissue_batch_set_launch")

    def set_chi_mode(self, mode: int):
        _check(lib.tissue_batch_set_chi_mode(self.handle, int(mode)), "tissue_batch_set_chi_mode")

    def set_graph_chunk(self, steps: int):
        _check(lib.tissue_batch_set_graph_chunk(self.handle, int(steps)), "tissue_batch_set_graph_chunk")

    def set_refill(self, min_idle_lanes: int):
        _check(lib.tissue_batch_set_refill(self.handle, int(min_idle_lanes)), "tissue_batch_set_refill")

    def set_whole_run(self, enable: bool):
        _check(lib.tissue_batch_set_whole_run(self.handle, int(bool(enable))), "tissue_batch_set_whole_run")

    def runs_whole(self) -> bool:
        rc = lib.tissue_batch_runs_whole(self.handle)
        _check(min(rc, 0), "tissue_batch_runs_whole")
        return rc == 1

    def set_regroup(self, mode: int):
        _check(lib.tissue_batch_set_regroup(self.handle, int(mode)), "tissue_batch_set_regroup")

    def restart(self, sim_ids=None, start_step: int = 0):
        for i, t in enumerate(self.tissues):
            t.restart(t.problem["sim_id"] if sim_ids is None else sim_ids[i], start_step)

    def sync(self):
        _check(lib.tissue_batch_sync(self.handle), "tissue_batch_sync")

    def set_members(self, tissues):
        """Replace the members in place (no host synchronisation); raises
        TissueError with code EBUSY when they do not fit the buffer."""
        tissues = list(tissues)
        arr = (C.c_void_p * max(len(tissues), 1))(*[t.handle.value for t in tissues])
        _check(lib.tissue_batch_set_members(self.handle, arr, len(tissues)), "tissue_batch_set_members")
        self.tissues = tissues
        self._arr = arr

    def close(self):
        if getattr(self, "handle", None):
            lib.tissue_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
