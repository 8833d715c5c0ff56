"""Shared helpers of the GPU tests: run the HIP path and the oracle on the
same seeded problem and compare."""
import numpy as np

from paper_1806_10889_amd import workloads as W


def gpu_run(problem, n_steps, trace=False, persistent=None, wpc=0, graph_chunk=None, chunks=None,
            allow_flags=False, chi_mode=None, jit=True, regroup=None, whole_run=False):
    """The tissue stepped through the library.  whole_run=False (the
    default here) keeps the step-by-step launches these tests exercise; the
    whole-run kernel of small tissues has tests of its own."""
    from paper_1806_10889_amd import tissue as T
    t = T.Tissue(problem, trace_steps=n_steps if trace else 0, jit=jit)
    assert t.stats()["jit"] == int(jit), "network kernels not compiled"
    t.set_whole_run(whole_run)
    if chi_mode is not None:
        t.set_chi_mode(chi_mode)
    if regroup is not None:
        t.set_regroup(regroup)
    if persistent is not None:
        t.set_launch(persistent, wpc)
    if graph_chunk is not None:
        t.set_graph_chunk(graph_chunk)
    for c in (chunks or [n_steps]):
        t.step(problem["dt"], c)
    out = dict(counts=t.read_counts(allow_flags=allow_flags), stats=t.stats())
    if trace:
        s0 = int(problem.get("start_step", 0))
        out["trace"] = t.trace(s0, n_steps)
    t.close()
    return out


def assert_same(g, o, trace=True):
    assert np.array_equal(g["counts"], o.counts), \
        f"counts differ at {np.flatnonzero(g['counts'] != o.counts)[:10]}"
    assert g["stats"]["chi_events"] == o.chi_events
    assert g["stats"]["s_events"] == o.s_events
    assert g["stats"]["draws"] == o.draws
    if trace:
        ce, ct, se, st = g["trace"]
        assert np.array_equal(ce, o.chi_trace_events)
        assert np.array_equal(ct, o.chi_trace_t)
        if se.shape[1] == 0:
            # no S operator: the library has no edges; the oracle's edge trace is all zero
            assert not o.s_trace_events.any() and not o.s_trace_t.any()
        else:
            assert np.array_equal(se, o.s_trace_events)
            assert np.array_equal(st, o.s_trace_t)


def notch_uneven(seed, lattice, scheme="lie", n_steps=5):
    """The paper's network on cells of 1..4 x 1..4 voxels (face groups of
    different sizes on the two sides of an edge), Delta and NICD scattered,
    one promoter per cell."""
    rng = np.random.default_rng(seed)
    nx, ny = 6, 5
    w = rng.integers(1, 5, size=nx * ny)
    h = rng.integers(1, 5, size=nx * ny)
    nvox = int((w * h).sum())
    x0 = np.zeros((nvox, 4), np.int32)
    x0[:, 0] = rng.integers(0, 30, nvox)
    x0[:, 1] = rng.integers(0, 5, nvox)
    off = np.concatenate([[0], np.cumsum(w * h)[:-1]])
    x0[off, 2] = 1
    p = W.make_problem(W.model_notch_paper(), lattice=lattice, nx=nx, ny=ny, mesh_w=w, mesh_h=h,
                       rates=[100.0, 64.0, 25.0, 1.0, 1.0], trans_rate=2.0,
                       diffusion=[16.0, 16.0, 0.0, 0.0], init_counts=x0, seed=seed, dt=0.05,
                       n_steps=n_steps)
    p["scheme"] = scheme
    return p
