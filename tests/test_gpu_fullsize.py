"""GPU parity at the sizes the benchmark runs, in the launch shapes it times.

Every test compares the HIP path (through the C-ABI) with the CPU FP64 oracle
element by element: counts, event and draw totals, and, where traced, the
per-(cell, step) and per-(edge, step) event counts and last-event-time bits.

* the 64x64 headline tissue over its first 50 splitting steps (persistent and
  one-workgroup-per-item launches, graphs), and over its whole horizon of
  2000 steps in the benchmark's launch configuration (final counts and
  totals);
* the uneven 256x256 tissue over its first 20 steps in the automatic layout
  with forked graph branches: compact classes of 35 975 and 20 217 cells
  regrouped by load in segments of at most 16 384 cells, and the row head of
  its 64-leaf class;
* a forced-compact class of 22 500 cells (two regroup segments) and a 64-leaf
  class of 18 496 cells whose row head is cut from a segmented class;
* the full 512-tissue batch exactly as the batched leg builds it, with 16
  sampled tissues (the 8 smallest and 8 at random) against the oracle over
  the first 5 steps (graphs of 2) and over the whole horizon of 200 steps;
* the serving loop at four lanes on the serving workload's own requests:
  32 sampled results equal the same requests run alone, 8 equal the oracle.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same, gpu_run
from paper_1806_10889_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def config2_50(oracle_lib):
    p = W.config2(n_steps=50)
    print("oracle: hex 64x64, 4x4 cells, 50 steps", flush=True)
    return p, oracle_lib.run(p, p["dt"], 50, trace=True)


@pytest.mark.parametrize("persistent,chunk", [(1, 25), (0, 50), (1, 0)])
def test_config2_full_first_50_steps(config2_50, persistent, chunk):
    """The headline workload's first 50 steps in the automatic layout (rows
    of 16 lanes): persistent grids or one workgroup per item, replayed from
    graphs of 25 or 50 steps, or eager."""
    p, o = config2_50
    g = gpu_run(p, 50, trace=True, persistent=persistent, graph_chunk=chunk, chi_mode=2)
    assert_same(g, o)


def test_config3_full_auto_forked_graphs(oracle_lib):
    """The uneven 256x256 tissue as the benchmark runs it (automatic layout,
    one workgroup per item, regroup automatic): the 16- and 32-leaf classes
    compact and regrouped in 3 and 2 segments, the 64-leaf class's heaviest
    1024 cells in rows, every class a parallel branch of the step graph;
    its first 20 steps (three graphs of 6 and an eager tail) on every cell
    and edge."""
    from paper_1806_10889_amd import tissue as T
    p = W.config3(n_steps=20)
    P = [1 << int(np.ceil(np.log2(w * h))) for w, h in zip(p["mesh_w"], p["mesh_h"])]
    classes = {k: P.count(k) for k in set(P)}
    assert classes[16] > 2 * 16384 and 16384 < classes[32] <= 2 * 16384 and classes[64] > 4096
    print("oracle: hex 256x256 uneven, 20 steps", flush=True)
    o = oracle_lib.run(p, p["dt"], 20, trace=True)
    t = T.Tissue(p, trace_steps=20)
    t.set_chi_mode(2)
    t.set_regroup(2)
    t.set_launch(False, 0)
    t.set_graph_chunk(6)
    t.step(p["dt"], 20)
    g = dict(counts=t.read_counts(), stats=t.stats(), trace=t.trace(0, 20))
    t.close()
    assert_same(g, o)


@pytest.mark.parametrize("persistent", [False, True])
def test_regroup_segments_of_a_large_compact_class(oracle_lib, persistent):
    """150x150 cells of 4x4 voxels in the compact layout with the regroup
    forced on: the class's 22 500 cells are reordered in two segments
    (16 384 + 6 116), each rewritten in place; 4 steps in graphs of 2 (forked
    branches or persistent grids), every cell against the oracle."""
    p = W.config2(side=150, n_steps=4)
    print("oracle: hex 150x150, 4x4 cells, 4 steps", flush=True)
    o = oracle_lib.run(p, p["dt"], 4, trace=True)
    g = gpu_run(p, 4, trace=True, persistent=persistent, graph_chunk=2, chi_mode=3, regroup=1)
    assert_same(g, o)


def test_row_head_cut_from_a_segmented_class(oracle_lib):
    """136x136 cells of 8x8 voxels, automatic layout: the 64-leaf class of
    18 496 cells is compact, regrouped in two segments, and its heaviest 1024
    cells run in rows of 64 lanes; forked graphs of 2 steps and an eager
    step, every cell against the oracle."""
    rng = np.random.default_rng(151)
    m = W.model_nd5()
    side = 136
    x0 = rng.integers(0, 51, size=(side * side * 64, 5)).astype(np.int32)
    p = W.make_problem(m, lattice=1, nx=side, ny=side, mesh_w=8, mesh_h=8,
                       rates=10.0 ** rng.uniform(-2, 1, m["n_reactions"]), trans_rate=0.8,
                       diffusion=1.0, init_counts=x0, seed=151, dt=0.02, n_steps=3)
    print("oracle: hex 136x136, 8x8 cells, 3 steps", flush=True)
    o = oracle_lib.run(p, p["dt"], 3, trace=True)
    g = gpu_run(p, 3, trace=True, persistent=False, graph_chunk=2, chi_mode=2, regroup=2)
    assert_same(g, o)


def test_config2_full_horizon(oracle_lib):
    """The headline workload over its whole horizon (2000 steps, about
    1.5e9 events) in the benchmark's launch configuration (rows of 16
    lanes, one workgroup per item, graphs of 25 steps): the final counts
    of every voxel and the event and draw totals equal the oracle's."""
    p = W.config2()
    print("oracle: hex 64x64, 4x4 cells, 2000 steps", flush=True)
    o = oracle_lib.run(p, p["dt"], 2000)
    g = gpu_run(p, 2000, persistent=0, graph_chunk=25, chi_mode=1)
    assert_same(g, o, trace=False)


def test_config4_full_horizon_sampled(oracle_lib):
    """The 512-tissue sweep over its whole horizon (200 steps) as the
    batched leg runs it (one Batch, automatic layout and regroup, the
    default persistent launch and graphs); the same 16 sampled tissues (the
    8 smallest and 8 at random) against the oracle."""
    from paper_1806_10889_amd import tissue as T
    probs = W.config4()
    n = probs[0]["n_steps"]
    ts = [T.Tissue(p) for p in probs]
    b = T.Batch(ts)
    b.set_regroup(2)
    b.step(probs[0]["dt"], n)
    b.sync()
    sizes = np.array([p["nx"] * p["ny"] for p in probs])
    rng = np.random.default_rng(404)
    small = list(np.argsort(sizes, kind="stable")[:8])
    rest = [i for i in range(len(probs)) if i not in small]
    sample = small + list(rng.choice(rest, size=8, replace=False))
    for i in sample:
        print(f"oracle: batch member {i} ({probs[i]['nx']}x{probs[i]['ny']}), {n} steps", flush=True)
        o = oracle_lib.run(probs[i], probs[i]["dt"], n)
        st = ts[i].stats()
        assert np.array_equal(ts[i].read_counts(), o.counts), i
        assert (st["chi_events"], st["s_events"], st["draws"]) == (o.chi_events, o.s_events, o.draws)
    b.close()
    for t in ts:
        t.close()


def test_config4_full_batch_sampled(oracle_lib):
    """The 512-tissue sweep (3.1 M cells) built exactly as the batched leg
    builds it (one Batch, automatic layout and regroup, the default
    persistent launch), stepped 5 times in graphs of 2 steps and an eager
    step; 16 tissues (the 8 smallest and 8 at random) against the oracle."""
    from paper_1806_10889_amd import tissue as T
    probs = W.config4(n_steps=5)
    ts = [T.Tissue(p) for p in probs]
    b = T.Batch(ts)
    b.set_regroup(2)
    b.set_graph_chunk(2)
    b.step(probs[0]["dt"], 5)
    b.sync()
    sizes = np.array([p["nx"] * p["ny"] for p in probs])
    rng = np.random.default_rng(404)
    small = list(np.argsort(sizes, kind="stable")[:8])
    rest = [i for i in range(len(probs)) if i not in small]
    sample = small + list(rng.choice(rest, size=8, replace=False))
    for i in sample:
        print(f"oracle: batch member {i} ({probs[i]['nx']}x{probs[i]['ny']})", flush=True)
        o = oracle_lib.run(probs[i], probs[i]["dt"], 5)
        st = ts[i].stats()
        assert np.array_equal(ts[i].read_counts(), o.counts), i
        assert (st["chi_events"], st["s_events"], st["draws"]) == (o.chi_events, o.s_events, o.draws)
    b.close()
    for t in ts:
        t.close()


def test_serving_four_lanes_alone_equals_mix(oracle_lib):
    """The serving loop at the benchmark's four lanes on the serving
    workload's own requests (hex tissues of 16..16384 cells, 1..16 voxels
    per cell), arrivals replayed in real time at 200 per second with the
    HBM budget binding: 32 sampled results equal the same request run alone
    on the device, 8 of them equal the oracle."""
    from paper_1806_10889_amd import serve
    from paper_1806_10889_amd import tissue as T
    reqs = serve.requests_from_workload(96, rate_hz=200.0, n_steps=30)
    be = serve.GpuBackend(lanes=4)
    need = [be.required_bytes(r.problem) for r in reqs]
    budget = max(max(need), sum(need) // 6)
    srv = serve.Server(be, max_bytes=budget, max_active=4096, quantum=10, keep_results=True)
    st, done = srv.run(reqs, real_time=True)
    assert st.completed == len(reqs) and st.max_active > 4 and st.max_bytes <= budget
    by_id = {r.rid: r for r in done}
    rng = np.random.default_rng(505)
    sample = sorted(rng.choice(len(reqs), size=32, replace=False))
    for q in sample:
        r = by_id[q]
        t = T.Tissue(r.problem)
        t.step(r.problem["dt"], r.n_steps)
        assert np.array_equal(r.result, t.read_counts()), q
        st1 = t.stats()
        assert r.events == st1["chi_events"] + st1["s_events"], q
        t.close()
    for q in sample[::4]:
        r = by_id[q]
        print(f"oracle: request {q} ({r.problem['nx']}x{r.problem['ny']})", flush=True)
        o = oracle_lib.run(r.problem, r.problem["dt"], r.n_steps)
        assert np.array_equal(r.result, o.counts), q
