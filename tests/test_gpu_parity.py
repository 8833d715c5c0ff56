"""GPU parity: the HIP path (through the C-ABI) against the CPU FP64 oracle.

Bit-exact on every integer count, on the per-(cell, step) and per-(edge,
step) event counts and on the bits of each unit-step's last event time, and
on the event/draw totals.  Sizes span several work items and ragged tails;
the last tests run the full-size workloads for a few steps in the launch
configuration the benchmark times.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same, gpu_run, notch_uneven as _notch_uneven
from paper_1806_10889_amd import workloads as W

pytestmark = pytest.mark.gpu


def _oracle(oracle_lib, p, n, trace=True, **kw):
    return oracle_lib.run(p, p["dt"], n, trace=trace, **kw)


# chi kernel: one lane per cell / one 16-lane row per cell / the compact
# layout (1, 2 or 4 lanes per cell) / rows of 32 lanes for the small cells
MODES = [0, 1, 3, 4]


@pytest.mark.parametrize("mode", MODES)
def test_config1_full_horizon(oracle_lib, mode):
    p = W.config1()
    o = _oracle(oracle_lib, p, p["n_steps"])
    g = gpu_run(p, p["n_steps"], trace=True, chi_mode=mode)
    assert o.chi_events > 1000
    assert_same(g, o)


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mode", MODES)
def test_config2_reduced(oracle_lib, mode, jit):
    p = W.config2(side=9, n_steps=12)  # 81 cells: two chi items, ragged S tail
    o = _oracle(oracle_lib, p, 12)
    g = gpu_run(p, 12, trace=True, chi_mode=mode, jit=jit)
    assert o.chi_events > 10000 and o.s_events > 1000
    assert_same(g, o)


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("lattice", [0, 1])
def test_uneven_meshes_overlapping_faces(oracle_lib, lattice, mode, jit):
    p = W.random_problem(31 + lattice, lattice=lattice, nx=9, ny=7, model="nd5", uneven=True,
                         dt=0.05, n_steps=6)
    o = _oracle(oracle_lib, p, 6)
    g = gpu_run(p, 6, trace=True, chi_mode=mode, jit=jit)
    assert o.s_events > 0
    assert_same(g, o)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("mesh", [(1, 1), (2, 2), (2, 1), (3, 5), (8, 8), (7, 3), (1, 8), (4, 4),
                                  (2, 8), (5, 5), (5, 7), (6, 6), (8, 4)])
def test_mesh_shapes(oracle_lib, mesh, mode):
    p = W.random_problem(40 + mesh[0] * 8 + mesh[1], lattice=1, nx=5, ny=4, model="nd5",
                         mesh=mesh, dt=0.05, n_steps=4)
    o = _oracle(oracle_lib, p, 4)
    assert_same(gpu_run(p, 4, trace=True, chi_mode=mode), o)


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("model", ["nd5", "nd4", "bd", "dimer", "diff", "tr"])
def test_networks(oracle_lib, model, mode, jit):
    """Compiled-network and generic kernels on other table sizes: 4 species /
    7 reactions, 1 species / 2 reactions, order-2 same-species, diffusion
    only, signalling only."""
    p = W.random_problem(51, lattice=0, nx=7, ny=6, model=model, mesh=(3, 3), dt=0.1,
                         n_steps=5, rate_lo=-1.0, rate_hi=1.0)
    o = _oracle(oracle_lib, p, 5)
    assert_same(gpu_run(p, 5, trace=True, chi_mode=mode, jit=jit), o)


@pytest.mark.parametrize("mode", MODES)
def test_nd4_well_mixed_square(oracle_lib, mode):
    p = W.random_problem(50, lattice=0, nx=13, ny=11, model="nd4", mesh=(1, 1), dt=0.1,
                         n_steps=20, rate_lo=-1.0, rate_hi=1.0)
    o = _oracle(oracle_lib, p, 20)
    assert_same(gpu_run(p, 20, trace=True, chi_mode=mode), o)


@pytest.mark.parametrize("persistent,wpc,chunk,mode", [(0, 0, 0, 0), (1, 0, 0, 1), (1, 1, 0, 2),
                                                       (1, 3, 2, 0), (0, 0, 3, 1), (1, 8, 5, 2),
                                                       (1, 0, 0, 3), (0, 0, 4, 3)])
def test_launch_shapes_do_not_change_bits(oracle_lib, persistent, wpc, chunk, mode):
    p = W.random_problem(60, lattice=1, nx=11, ny=10, model="nd5", uneven=True, dt=0.05,
                         n_steps=7)
    o = _oracle(oracle_lib, p, 7)
    g = gpu_run(p, 7, trace=True, persistent=persistent, wpc=wpc, graph_chunk=chunk, chi_mode=mode)
    assert_same(g, o)


def test_chunking_restart_and_resume(oracle_lib):
    from paper_1806_10889_amd import tissue as T
    p = W.random_problem(70, lattice=1, nx=8, ny=8, model="nd5", mesh=(4, 4), dt=0.05, n_steps=9)
    o = _oracle(oracle_lib, p, 9, trace=False)
    g = gpu_run(p, 9, chunks=[2, 3, 4])
    assert np.array_equal(g["counts"], o.counts)
    t = T.Tissue(p)
    t.set_graph_chunk(2)
    t.step(p["dt"], 9)
    a = t.read_counts()
    t.restart(p["sim_id"], 0)
    t.step(p["dt"], 9)
    assert np.array_equal(t.read_counts(), a)
    assert np.array_equal(a, o.counts)
    # resume from a snapshot: run 4, snapshot, new tissue from step 4
    t.restart(p["sim_id"], 0)
    t.step(p["dt"], 4)
    snap = t.read_counts()
    q = dict(p, init_counts=snap.reshape(p["init_counts"].shape), start_step=4)
    t2 = T.Tissue(q)
    t2.step(p["dt"], 5)
    assert np.array_equal(t2.read_counts(), o.counts)
    # another sim_id is another stream
    t.restart(p["sim_id"] + 1, 0)
    t.step(p["dt"], 9)
    other = t.read_counts()
    o2 = oracle_lib.run(dict(p, sim_id=p["sim_id"] + 1), p["dt"], 9)
    assert np.array_equal(other, o2.counts) and not np.array_equal(other, a)


def test_batch_equals_plain_and_oracle(oracle_lib):
    from paper_1806_10889_amd import tissue as T
    probs = [
        W.random_problem(80, lattice=1, nx=9, ny=9, model="nd5", mesh=(4, 4), dt=0.05, sim_id=3),
        W.random_problem(81, lattice=1, nx=5, ny=7, model="nd5", uneven=True, dt=0.05, sim_id=4),
        W.random_problem(82, lattice=0, nx=6, ny=4, model="nd4", mesh=(1, 1), dt=0.05, sim_id=5),
        W.random_problem(83, lattice=0, nx=3, ny=3, model="nd5", mesh=(2, 3), dt=0.05, sim_id=6),
        W.random_problem(84, lattice=1, nx=1, ny=1, model="nd5", mesh=(4, 4), dt=0.05, sim_id=7),
        W.random_problem(85, lattice=1, nx=4, ny=4, model="bd", mesh=(1, 1), dt=0.05, sim_id=8),
    ]
    probs[3]["start_step"] = 17
    n = 6
    ts = [T.Tissue(p, jit=(i % 2 == 0)) for i, p in enumerate(probs)]  # mixed kernels in one batch
    b = T.Batch(ts)
    b.step(0.05, 2)
    b.set_launch(False)
    b.set_chi_mode(1)
    b.step(0.05, 3)
    b.set_chi_mode(0)
    b.step(0.05, 1)
    b.sync()
    for p, t in zip(probs, ts):
        o = oracle_lib.run(p, 0.05, n)
        assert np.array_equal(t.read_counts(), o.counts), p["name"]
        st = t.stats()
        assert (st["chi_events"], st["s_events"], st["draws"]) == (o.chi_events, o.s_events, o.draws)
        assert st["steps_done"] == p["start_step"] + n


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_compact_wide_cells_with_redo(oracle_lib, persistent):
    """A batch of uneven-mesh tissues in the compact layout (1, 2 and 4
    lanes per cell), regrouped by load before every launch: every member's
    cells of a class share one launch, and
    cells of several members and classes reach 2^16 and are redone from
    their launch's part of the redo list; graphs of 2 steps (classes as
    parallel branches with one workgroup per item, or persistent grids);
    every member against the oracle."""
    from paper_1806_10889_amd import tissue as T
    probs = [W.random_problem(120 + k, lattice=k % 2, nx=6, ny=5, model="nd5", uneven=True,
                              dt=0.05, sim_id=10 + k, n_steps=4) for k in range(4)]
    for k, p in enumerate(probs):
        sz = p["mesh_w"].astype(np.int64) * p["mesh_h"]
        off = np.concatenate([[0], np.cumsum(sz)])
        big = np.flatnonzero(sz > 16)[:2]
        small = np.flatnonzero(sz <= 16)[:1]
        for c in list(big) + list(small):
            p["init_counts"][off[c + 1] - 1 - k % 3, 0] = 65535
    ts = [T.Tissue(p) for p in probs]
    b = T.Batch(ts)
    b.set_chi_mode(3)
    b.set_regroup(1)  # the load-ordered regroup before every compact launch
    b.set_launch(persistent)
    b.set_graph_chunk(2)
    b.step(0.05, 4)
    b.sync()
    for p, t in zip(probs, ts):
        o = oracle_lib.run(p, 0.05, 4)
        assert np.array_equal(t.read_counts(), o.counts), p["name"]
        st = t.stats()
        assert (st["chi_events"], st["s_events"], st["draws"]) == (o.chi_events, o.s_events, o.draws)


@pytest.mark.parametrize("refill,regroup", [(0, 0), (1, 0), (8, 0), (8, 1), (33, 1), (64, 0)])
def test_lane_refill_uneven_loads(oracle_lib, refill, regroup):
    """The compact layout with lane refill in a persistent batch: a
    wavefront's idle lanes take the next cells of the launch, of other items
    and other tissues, while its busy lanes go on.  Tissues with loads that
    differ by more than an order of magnitude (rates scaled per tissue, a
    few hot cells with twenty times the molecules), cells of 4..16 voxels
    (1 lane each) next to larger ones (2 and 4 lanes, no refill), counts at
    2^16 redone at full width; graphs of 2 steps and an eager step; every
    member's counts, totals and per-cell traces against the oracle."""
    from paper_1806_10889_amd import tissue as T
    probs = []
    for k, (mesh, scale) in enumerate([((4, 4), 1.0), ((2, 3), 12.0), (None, 3.0), ((4, 4), 0.3),
                                        ((3, 3), 30.0)]):
        p = W.random_problem(160 + k, lattice=k % 2, nx=7 + k, ny=6, model="nd5", mesh=mesh,
                             uneven=mesh is None, dt=0.05, sim_id=20 + k, n_steps=5)
        p["rates"] = p["rates"] * scale
        V = p["mesh_w"].astype(np.int64) * p["mesh_h"]
        off = np.concatenate([[0], np.cumsum(V)])
        for c in (1, 9, 17):  # hot cells
            p["init_counts"][off[c]:off[c + 1]] *= 20
        p["init_counts"][off[5], 0] = 65535  # the redo at full width
        probs.append(p)
    ts = [T.Tissue(p, trace_steps=5) for p in probs]
    b = T.Batch(ts)
    b.set_chi_mode(3)
    b.set_regroup(regroup)
    b.set_refill(refill)
    b.set_graph_chunk(2)
    b.step(0.05, 5)
    b.sync()
    for p, t in zip(probs, ts):
        o = _oracle(oracle_lib, p, 5)
        assert_same(dict(counts=t.read_counts(), stats=t.stats(), trace=t.trace(0, 5)), o)
    b.close()
    with pytest.raises(T.TissueError) as ei:
        ts[0].set_refill(65)
    assert ei.value.code == T.EINVAL
    for t in ts:
        t.close()


@pytest.mark.parametrize("refill", [0, 8])
def test_step_timed_names_the_refill_kernel(oracle_lib, refill):
    """A persistent compact launch of 4x4 cells reports whether it ran with
    lane refill; same bits either way."""
    from paper_1806_10889_amd import tissue as T
    p = W.config2(side=40, n_steps=3)
    t = T.Tissue(p)
    t.set_chi_mode(3)
    t.set_launch(True, 0)
    t.set_refill(refill)
    tm = t.step_timed(p["dt"], 3)
    g = dict(counts=t.read_counts(), stats=t.stats())
    t.close()
    assert_same(g, _oracle(oracle_lib, p, 3, trace=False), trace=False)
    assert tm["chi_kernel"] == 3 and tm["chi_refill"] == int(refill > 0)


@pytest.mark.parametrize("scheme", ["lie", "strang"])
@pytest.mark.parametrize("persistent", [False, True])
def test_regroup_by_load_keeps_bits(oracle_lib, scheme, persistent):
    """The regroup pass before every compact launch (forced on) reorders
    each class's cells by load between chi passes; bits, per-cell traces
    and totals stay the oracle's, over graphs of 3 steps and an eager tail,
    with cells redone at full width."""
    p = W.random_problem(140, lattice=1, nx=11, ny=9, model="nd5", uneven=True, dt=0.05, n_steps=7)
    p["scheme"] = scheme
    off = np.concatenate([[0], np.cumsum(p["mesh_w"].astype(np.int64) * p["mesh_h"])])
    for c in (3, 40, 77):
        p["init_counts"][off[c], 0] = 65535
    o = _oracle(oracle_lib, p, 7)
    from paper_1806_10889_amd import tissue as T
    t = T.Tissue(p, trace_steps=7)
    t.set_chi_mode(3)
    t.set_regroup(1)
    t.set_launch(persistent)
    t.set_graph_chunk(3)
    t.step(p["dt"], 7)
    g = dict(counts=t.read_counts(), stats=t.stats(), trace=t.trace(0, 7))
    with pytest.raises(T.TissueError):
        t.set_regroup(3)
    t.close()
    assert_same(g, o)


@pytest.mark.parametrize("persistent", [False, True])
def test_row_head_of_the_largest_cells(oracle_lib, persistent):
    """Automatic layout on a single tissue of 4096 cells of 8x8 voxels: the
    64-leaf class is compact and regrouped by load, its heaviest 1024 cells
    running in rows of 64 lanes (a launch of their own, a parallel graph
    branch); same bits as the oracle."""
    rng = np.random.default_rng(150)
    m = W.model_nd5()
    x0 = rng.integers(0, 51, size=(64 * 64 * 64, 5)).astype(np.int32)
    p = W.make_problem(m, lattice=1, nx=64, ny=64, mesh_w=8, mesh_h=8,
                       rates=10.0 ** rng.uniform(-2, 1, m["n_reactions"]), trans_rate=0.8,
                       diffusion=1.0, init_counts=x0, seed=150, dt=0.02, n_steps=3)
    o = _oracle(oracle_lib, p, 3, threads=0)
    g = gpu_run(p, 3, trace=True, persistent=persistent, graph_chunk=2, chi_mode=2)
    assert_same(g, o)


@pytest.mark.parametrize("mode", [2, 3, 0])
def test_config4_sampled_tissues(oracle_lib, mode):
    from paper_1806_10889_amd import tissue as T
    probs = W.config4(n_tissues=40, side_hi=24, n_steps=5)
    ts = [T.Tissue(p) for p in probs]
    b = T.Batch(ts)
    b.set_chi_mode(mode)
    b.step(probs[0]["dt"], 5)
    b.sync()
    sizes = np.array([p["nx"] for p in probs])
    sample = list(np.argsort(sizes)[:4]) + [5, 17, 29, 39]
    for i in sample:
        o = oracle_lib.run(probs[i], probs[i]["dt"], 5)
        assert np.array_equal(ts[i].read_counts(), o.counts), i


def test_edge_cases(oracle_lib):
    from paper_1806_10889_amd import tissue as T
    # one cell: no edges
    p = W.random_problem(90, lattice=1, nx=1, ny=1, model="nd5", mesh=(3, 3), dt=0.05)
    assert_same(gpu_run(p, 3, trace=True), _oracle(oracle_lib, p, 3))
    # everything zero: no event, no draw
    p = W.random_problem(91, lattice=0, nx=3, ny=2, model="nd5", mesh=(2, 2), dt=0.05)
    p["init_counts"][:] = 0
    p["rates"][[0, 2]] = 0.0
    g = gpu_run(p, 3, trace=True)
    assert g["stats"]["draws"] == 0 and np.all(g["counts"] == 0)
    assert_same(g, _oracle(oracle_lib, p, 3))
    # S disabled
    p = W.random_problem(92, lattice=1, nx=4, ny=3, model="nd5", mesh=(4, 4), dt=0.05)
    p["trans_n"] = -1
    g = gpu_run(p, 3, trace=True)
    assert g["stats"]["s_events"] == 0
    assert_same(g, _oracle(oracle_lib, p, 3))
    # event cap: both stop the unit-step at the cap and flag it
    p = W.birth_death(5e4, 0.0, 0, nx=3, ny=2, dt=1.0)
    p["event_cap"] = 777
    o = oracle_lib.run(p, 1.0, 2)
    assert o.capped
    t = T.Tissue(p)
    t.step(1.0, 2)
    with pytest.raises(T.TissueError) as ei:
        t.read_counts()
    assert ei.value.code == T.ELIMIT
    assert np.array_equal(t.read_counts(allow_flags=True), o.counts)
    # overflow: a count crosses 2^26
    p = W.birth_death(50.0, 0.0, (1 << 26) - 5, nx=2, ny=1, dt=1.0)
    o = oracle_lib.run(p, 1.0, 1)
    assert o.overflow
    t = T.Tissue(p)
    t.step(1.0, 1)
    with pytest.raises(T.TissueError) as ei:
        t.read_counts()
    assert ei.value.code == T.EOVERFLOW
    assert np.array_equal(t.read_counts(allow_flags=True), o.counts)


def _range_problem():
    """4 cells of 4x4 voxels, one voxel per cell starting 5 below 2^26 and
    receiving A at rate 50 over two unit steps.  (No count can go negative:
    tissue creation rejects a reaction that removes a species it does not
    read.)"""
    net = W._net(["A", "B"], [("make", [], {"A": 1}), ("turn", ["A"], {"B": 1})], None)
    x0 = np.zeros((4 * 16, 2), np.int32)
    x0[:, 1] = 2
    x0[::16, 0] = (1 << 26) - 5
    return W.make_problem(net, lattice=1, nx=2, ny=2, mesh_w=4, mesh_h=4, rates=[50.0, 1e-9],
                          trans_rate=0.0, diffusion=[0.0, 1.0], init_counts=x0, seed=17,
                          dt=1.0, n_steps=2, name="range")


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mode", MODES)
def test_count_range_flag_in_every_layout(oracle_lib, mode, jit):
    """The range check in every chi layout (an OR of the integer counts
    against the power-of-two limit): a count crossing 2^26 (in the compact
    layout after the redo of its 16-bit counts) flags the tissue, with the
    oracle's counts and events."""
    from paper_1806_10889_amd import tissue as T
    p = _range_problem()
    o = _oracle(oracle_lib, p, 2, trace=False)
    assert o.overflow
    assert_same(gpu_run(p, 2, chi_mode=mode, jit=jit, allow_flags=True), o, trace=False)
    t = T.Tissue(p, jit=jit)
    t.set_chi_mode(mode)
    t.step(1.0, 2)
    with pytest.raises(T.TissueError) as ei:
        t.read_counts()
    assert ei.value.code == T.EOVERFLOW
    t.close()


@pytest.mark.parametrize("mesh", [(4, 4), (8, 4), (8, 8)])
@pytest.mark.parametrize("mode", MODES)
def test_event_cap_in_every_layout(oracle_lib, mode, mesh):
    """Cells of 16, 32 and 64 voxels (the compact layout with 1, 2 and 4
    lanes per cell) reach the event cap in every unit step: every layout
    stops each cell-step at the cap and flags the tissue, with the oracle's
    counts and events."""
    from paper_1806_10889_amd import tissue as T
    w, h = mesh
    net = W._net(["A", "B"], [("make", [], {"A": 1}), ("turn", ["A"], {"B": 1})], None)
    p = W.make_problem(net, lattice=1, nx=2, ny=2, mesh_w=w, mesh_h=h, rates=[20.0, 0.5],
                       trans_rate=0.0, diffusion=[1.0, 0.5], init_counts=np.zeros((4 * w * h, 2), np.int32),
                       seed=23, dt=1.0, n_steps=2, event_cap=500, name="cap")
    o = _oracle(oracle_lib, p, 2, trace=True)
    assert o.capped and (o.chi_trace_events == 500).all()
    assert_same(gpu_run(p, 2, trace=True, chi_mode=mode, allow_flags=True), o)
    t = T.Tissue(p)
    t.set_chi_mode(mode)
    t.step(1.0, 2)
    with pytest.raises(T.TissueError) as ei:
        t.read_counts()
    assert ei.value.code == T.ELIMIT
    t.close()


def test_invalid_calls_enqueue_nothing():
    from paper_1806_10889_amd import tissue as T
    p = W.random_problem(93, lattice=1, nx=3, ny=3, model="nd5", mesh=(2, 2), dt=0.05)
    t = T.Tissue(p)
    for dt, n in [(0.0, 1), (-1.0, 1), (float("nan"), 1), (float("inf"), 1), (0.1, -1)]:
        with pytest.raises(T.TissueError) as ei:
            t.step(dt, n)
        assert ei.value.code == T.EINVAL
    assert t.stats()["steps_done"] == 0
    assert np.array_equal(t.read_counts(), p["init_counts"].ravel())
    with pytest.raises(T.TissueError):
        t.trace(0, 1)  # created without trace
    with pytest.raises(T.TissueError):
        T.Tissue(dict(p, sim_id=1 << 30))


def test_batch_membership_rules():
    """A tissue twice in one batch is refused (its cells would run twice in
    one launch, racing on its counts), and a member cannot be destroyed
    while its batch lives; neither call enqueues work.  A step count that
    would carry the step index past 2^32 is refused by the timed step too."""
    from paper_1806_10889_amd import tissue as T
    p = W.random_problem(94, lattice=1, nx=3, ny=3, model="nd5", mesh=(2, 2), dt=0.05)
    a, b = T.Tissue(p), T.Tissue(dict(p, sim_id=1))
    with pytest.raises(T.TissueError) as ei:
        T.Batch([a, b, a])
    assert ei.value.code == T.EINVAL
    bt = T.Batch([a, b])
    with pytest.raises(T.TissueError) as ei:
        a.close()
    assert ei.value.code == T.ESTATE and a.handle is not None
    bt.step(0.05, 2)
    bt.close()
    a.close()
    assert b.stats()["steps_done"] == 2
    t = T.Tissue(dict(p, start_step=(1 << 32) - 3))
    with pytest.raises(T.TissueError) as ei:
        t.step_timed(0.05, 3)
    assert ei.value.code == T.EINVAL and t.stats()["steps_done"] == (1 << 32) - 3
    t.step_timed(0.05, 2)
    assert t.stats()["steps_done"] == (1 << 32) - 1
    t.close()
    b.close()


def test_batch_set_members_in_place(oracle_lib):
    """Continuous batching: members admitted and retired between steps of one
    batch (tissue_batch_set_members, no new batch), each tissue's bits equal
    to its steps alone; a member set over the batch's buffer answers EBUSY
    and changes nothing; a retired member can be destroyed; an empty batch
    steps nothing."""
    from paper_1806_10889_amd import tissue as T
    probs = [W.random_problem(170 + k, lattice=k % 2, nx=5 + 2 * k, ny=6, model="nd5",
                              mesh=(4, 4) if k % 3 else (2, 3), dt=0.05, sim_id=30 + k, n_steps=6)
             for k in range(5)]
    ts = [T.Tissue(p) for p in probs]
    b = T.Batch(ts[:2], capacity_bytes=4 << 20)
    b.step(0.05, 2)                      # 0, 1: steps 0..1
    b.set_members([ts[0], ts[1], ts[2]])
    b.step(0.05, 2)                      # 0, 1: 2..3; 2: 0..1
    b.set_members([ts[2], ts[3]])        # 0 and 1 retire
    ts[1].close()
    b.step(0.05, 2)                      # 2: 2..3; 3: 0..1
    b.set_members([])
    b.step(0.05, 3)                      # nothing
    b.set_members([ts[4], ts[0], ts[2]])
    b.step(0.05, 2)                      # 4: 0..1; 0: 4..5; 2: 4..5
    b.sync()
    big = T.Tissue(W.birth_death(1.0, 0.1, 3, nx=400, ny=400, dt=0.05))  # > 4 MiB of work lists
    with pytest.raises(T.TissueError) as ei:
        b.set_members([ts[4], big])
    assert ei.value.code == T.EBUSY
    b.step(0.05, 1)                      # unchanged members: 4: 2; 0: 6; 2: 6
    b.sync()
    want = {0: 7, 2: 7, 3: 2, 4: 3}
    for k, n in want.items():
        o = _oracle(oracle_lib, probs[k], n, trace=False)
        st = ts[k].stats()
        assert np.array_equal(ts[k].read_counts(), o.counts), k
        assert (st["chi_events"], st["s_events"], st["draws"], st["steps_done"]) == \
            (o.chi_events, o.s_events, o.draws, n)
    b.close()
    big.close()
    for k in want:
        ts[k].close()


def test_config3_reduced_uneven(oracle_lib):
    p = W.config3(side=24, n_steps=3)
    o = _oracle(oracle_lib, p, 3)
    assert_same(gpu_run(p, 3, trace=True), o)


@pytest.mark.parametrize("mode", [2, 0])
def test_full_size_config2_bench_launch(oracle_lib, mode):
    """The 64x64 hex, 4x4-voxel workload at full size, persistent launches
    replayed from a captured graph (as the benchmark runs it, automatic
    kernel choice), two steps against the oracle on every cell."""
    p = W.config2()
    o = _oracle(oracle_lib, p, 2)
    g = gpu_run(p, 2, trace=True, persistent=1, graph_chunk=1, chi_mode=mode)
    assert_same(g, o)


def test_gpu_birth_death_ensemble_law():
    """GPU ensemble of 16384 independent well-mixed cells: birth-death
    transient law (mean, variance within 3 SE; KS after the randomised PIT)."""
    import math

    from scipy import stats

    import refmath
    k, gamma, x0, dt, n = 5.0, 0.5, 20, 0.1, 20
    p = W.birth_death(k, gamma, x0, nx=128, ny=128, dt=dt, n_steps=n, seed=99)
    x = gpu_run(p, n)["counts"].astype(np.int64)
    q = math.exp(-gamma * dt * n)
    mean = x0 * q + (k / gamma) * (1 - q)
    var = x0 * q * (1 - q) + (k / gamma) * (1 - q)
    assert abs(x.mean() - mean) < 3 * math.sqrt(var / x.size)
    pmf = np.convolve(stats.binom.pmf(np.arange(x0 + 1), x0, q),
                      stats.poisson.pmf(np.arange(120), (k / gamma) * (1 - q)))[:120]
    m4 = float(np.sum(pmf * (np.arange(120) - mean) ** 4))
    assert abs(x.var() - var) < 3 * math.sqrt((m4 - var ** 2) / x.size)
    assert refmath.discrete_ks_pvalue(x, pmf) > 0.01


@pytest.mark.parametrize("jit", [True, False])
def test_lane16_redo_of_wide_counts(oracle_lib, jit):
    """Cells whose counts reach 2^16 (during a step, or from the start) are
    redone at full width by the follow-up launch: same bits as the oracle."""
    p = W.random_problem(95, lattice=1, nx=9, ny=8, model="nd5", mesh=(4, 4), dt=0.05, n_steps=4)
    x = p["init_counts"].reshape(72, 16, 5)
    x[3, 5, 0] = 65530          # N of a voxel of cell 3 crosses 2^16 under production
    x[17, :, 0] = 65535
    x[40, 2, 4] = 70000         # starts above 2^16
    p["rates"][0] = 50.0
    o = _oracle(oracle_lib, p, 4)
    assert_same(gpu_run(p, 4, trace=True, chi_mode=3, jit=jit), o)


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mesh", [(5, 5), (8, 8), (5, 7)])
def test_compact_wide_cells_redo_of_wide_counts(oracle_lib, mesh, jit):
    """Cells of 17..64 voxels in the compact layout (2 or 4 lanes per cell):
    counts that reach 2^16 in a voxel held by any lane of the group (during
    a step, or from the start) hand the cell to the full-width redo; jumps
    cross the lanes' voxel ranges; same bits as the oracle."""
    w, h = mesh
    V = w * h
    p = W.random_problem(96 + V, lattice=1, nx=9, ny=8, model="nd5", mesh=mesh, dt=0.05,
                         n_steps=4)
    x = p["init_counts"].reshape(72, V, 5)
    x[3, V - 1, 0] = 65530       # the cell's last lane crosses 2^16 under production
    x[17, 16, 0] = 65534         # first voxel of the second lane
    x[40, 2, 4] = 70000          # starts above 2^16 in the first lane
    x[41, ::16, 1] = 65535       # the first voxel of every lane
    p["rates"][0] = 50.0
    o = _oracle(oracle_lib, p, 4)
    assert_same(gpu_run(p, 4, trace=True, chi_mode=3, jit=jit), o)


@pytest.mark.parametrize("mode,expect", [(0, 0), (1, 1), (3, 3), (2, 1), (4, 4)])
def test_step_timed_same_bits_and_reports_kernel(oracle_lib, mode, expect):
    """The eagerly launched, event-bracketed steps give the oracle's bits, one
    chi launch and the same S passes per step, and name the chi layout that ran (auto
    takes rows for a tissue with fewer than 16 lanes of compact work per SIMD)."""
    from paper_1806_10889_amd import tissue as T
    p = W.config2(side=9, n_steps=7)
    o = _oracle(oracle_lib, p, 7, trace=False)
    t = T.Tissue(p)
    t.set_chi_mode(mode)
    tm = t.step_timed(p["dt"], 7)
    g = dict(counts=t.read_counts(), stats=t.stats())
    t.close()
    assert_same(g, o, trace=False)
    assert tm["chi_kernel"] == expect and tm["chi_leaves"] == 16
    assert tm["chi_launches"] == 7 and tm["s_launches"] >= 7 and tm["s_launches"] % 7 == 0


def test_step_timed_names_the_dominant_class(oracle_lib):
    """On a tissue of 4x4 and 8x8 cells in the compact layout the 64-leaf
    class dominates the eager steps' device time, and the timing names it
    (compact mode, 64 leaves); same bits as the oracle."""
    from paper_1806_10889_amd import tissue as T
    p = W.random_problem(130, lattice=1, nx=12, ny=12, model="nd5", mesh=(4, 4), dt=0.05, n_steps=3)
    w = np.where(np.arange(144) % 4 == 0, 8, 4).astype(np.int32)
    nvox = int((w * w).sum())
    x0 = np.random.default_rng(130).integers(0, 51, size=(nvox, 5)).astype(np.int32)
    q = W.make_problem(W.model_nd5(), lattice=1, nx=12, ny=12, mesh_w=w, mesh_h=w, rates=p["rates"],
                       trans_rate=p["trans_rate"], diffusion=1.0, init_counts=x0, seed=130,
                       dt=0.05, n_steps=3)
    o = _oracle(oracle_lib, q, 3, trace=False)
    t = T.Tissue(q)
    t.set_chi_mode(3)
    tm = t.step_timed(q["dt"], 3)
    g = dict(counts=t.read_counts(), stats=t.stats())
    t.close()
    assert_same(g, o, trace=False)
    assert tm["chi_kernel"] == 3 and tm["chi_leaves"] == 64
    assert tm["chi_launches"] == 6
    assert 0 < tm["chi_ms"] <= tm["total_ms"] and 0 < tm["s_ms"] <= tm["total_ms"]


# ---------------------------------------------------------------------------
# Strang splitting: chi over dt/2 (tag 0), S over dt, chi over dt/2 (tag 2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mode", MODES)
def test_strang_config2_reduced(oracle_lib, mode, jit):
    p = W.config2(side=9, n_steps=10)
    p["scheme"] = "strang"
    o = _oracle(oracle_lib, p, 10)
    g = gpu_run(p, 10, trace=True, chi_mode=mode, jit=jit)
    assert o.chi_events > 10000 and o.s_events > 1000
    assert_same(g, o)


@pytest.mark.parametrize("mode", MODES)
def test_strang_uneven_overlapping_faces_and_redo(oracle_lib, mode):
    p = W.random_problem(33, lattice=1, nx=9, ny=7, model="nd5", uneven=True, dt=0.05, n_steps=6)
    p["scheme"] = "strang"
    o = _oracle(oracle_lib, p, 6)
    assert o.s_events > 0
    assert_same(gpu_run(p, 6, trace=True, chi_mode=mode, chunks=[2, 4]), o)
    q = W.random_problem(95, lattice=1, nx=9, ny=8, model="nd5", mesh=(4, 4), dt=0.05, n_steps=3)
    q["scheme"] = "strang"
    q["init_counts"].reshape(72, 16, 5)[17, :, 0] = 65535  # the compact layout redoes these
    assert_same(gpu_run(q, 3, trace=True, chi_mode=mode), _oracle(oracle_lib, q, 3))


def test_strang_batch_and_scheme_mismatch(oracle_lib):
    from paper_1806_10889_amd import tissue as T
    probs = [W.random_problem(60 + i, lattice=i % 2, nx=5 + i, ny=4, model="nd5",
                              mesh=(1 + i % 4, 2), dt=0.1, n_steps=5) for i in range(4)]
    for p in probs:
        p["scheme"] = "strang"
    ts = [T.Tissue(p) for p in probs]
    b = T.Batch(ts)
    b.step(0.1, 5)
    b.sync()
    for p, t in zip(probs, ts):
        o = _oracle(oracle_lib, p, 5, trace=False)
        assert_same(dict(counts=t.read_counts(), stats=t.stats()), o, trace=False)
    b.close()
    lie = dict(probs[0], scheme="lie", sim_id=99)
    t2 = T.Tissue(lie)
    with pytest.raises(T.TissueError, match="scheme"):
        T.Batch([ts[1], t2])
    t2.close()
    for t in ts:
        t.close()


def test_strang_step_timed_two_chi_launches_per_step(oracle_lib):
    from paper_1806_10889_amd import tissue as T
    p = W.config2(side=9, n_steps=4)
    p["scheme"] = "strang"
    t = T.Tissue(p)
    tm = t.step_timed(p["dt"], 4)
    g = dict(counts=t.read_counts(), stats=t.stats())
    t.close()
    assert_same(g, _oracle(oracle_lib, p, 4, trace=False), trace=False)
    assert tm["chi_launches"] == 8


# ---------------------------------------------------------------------------
# The paper's Notch model: first-order signalling into the facing voxel
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mode", MODES)
def test_notch_paper_model(oracle_lib, mode, jit):
    p = W.config_notch(side=7, n_steps=8)
    o = _oracle(oracle_lib, p, 8)
    assert o.s_events > 0 and o.chi_events > 10000
    assert_same(gpu_run(p, 8, trace=True, chi_mode=mode, jit=jit), o)


@pytest.mark.parametrize("scheme", ["lie", "strang"])
@pytest.mark.parametrize("lattice", [0, 1])
def test_notch_first_order_uneven_faces(oracle_lib, lattice, scheme):
    p = _notch_uneven(80 + lattice, lattice, scheme)
    o = _oracle(oracle_lib, p, 5)
    assert o.s_events > 100
    for mode in MODES:
        assert_same(gpu_run(p, 5, trace=True, chi_mode=mode), o)


def test_notch_and_trans_tissues_share_a_batch(oracle_lib):
    from paper_1806_10889_amd import tissue as T
    probs = [_notch_uneven(90, 0), W.config2(side=6, n_steps=5), _notch_uneven(91, 1)]
    ts = [T.Tissue(p) for p in probs]
    b = T.Batch(ts)
    b.step(probs[0]["dt"], 5)
    b.sync()
    for p, t in zip(probs, ts):
        o = _oracle(oracle_lib, p, 5, trace=False)
        assert_same(dict(counts=t.read_counts(), stats=t.stats()), o, trace=False)
    b.close()
    for t in ts:
        t.close()


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_classes_in_parallel_graph_branches(oracle_lib, scheme, jit):
    """One workgroup per item and captured graphs: the leaf-count classes'
    chi launches run as parallel graph branches; same bits as the oracle
    (uneven meshes: several classes, overlapping faces)."""
    p = W.random_problem(37, lattice=1, nx=9, ny=7, model="nd5", uneven=True, dt=0.05, n_steps=6)
    p["scheme"] = scheme
    o = _oracle(oracle_lib, p, 6)
    for mode in (0, 1, 2, 3, 4):
        g = gpu_run(p, 6, trace=True, persistent=False, graph_chunk=2, chi_mode=mode, jit=jit)
        assert_same(g, o)


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_compact_launches_with_redo_in_forked_graphs(oracle_lib, scheme):
    """Compact-layout launches of several leaf-count classes (1, 2 and 4
    lanes per cell), each handing cells back for the full-width redo, as
    parallel branches of the step graphs (each launch with its own queue
    words and part of the redo list); same bits as the oracle."""
    p = W.random_problem(39, lattice=0, nx=9, ny=7, model="nd5", uneven=True, dt=0.05, n_steps=4)
    p["scheme"] = scheme
    P = [1 << int(np.ceil(np.log2(w * h))) for w, h in zip(p["mesh_w"], p["mesh_h"])]
    off = np.concatenate([[0], np.cumsum(p["mesh_w"].astype(np.int64) * p["mesh_h"])])
    x = p["init_counts"]
    wide = {}
    for c, pc in enumerate(P):
        if wide.get(pc, 0) < 2:
            x[off[c + 1] - 1, 0] = 65535
            wide[pc] = wide.get(pc, 0) + 1
    assert len(wide) >= 5 and 32 in wide and 64 in wide
    o = _oracle(oracle_lib, p, 4)
    g = gpu_run(p, 4, trace=True, persistent=False, graph_chunk=2, chi_mode=3)
    assert_same(g, o)
