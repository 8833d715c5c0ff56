"""The whole-run kernel of small tissues (every step of a call in one
launch, the state in LDS): bit-exact against the CPU FP64 oracle --
counts, event and draw totals, per-(cell, step) and per-(edge, step) event
counts and last-event times -- for Lie and Strang splitting, trans and
first-order signalling, overlapping face groups (several S passes), calls
that cross the kernel's per-launch step bound, resumed runs, batches, and
the range and event-cap flags; and the rule that decides when it runs."""
import numpy as np
import pytest

from gpu_helpers import assert_same, gpu_run
from paper_1806_10889_amd import workloads as W

pytestmark = pytest.mark.gpu


def _cells(seed, lattice, n_steps, w, h, nx=6, ny=6):
    """The paper's network (first-order signalling) on cells of w x h
    voxels, Delta and NICD scattered, one promoter per cell."""
    rng = np.random.default_rng(seed)
    nvox = nx * ny * w * h
    x0 = np.zeros((nvox, 4), np.int32)
    x0[:, 0] = rng.integers(0, 30, nvox)
    x0[:, 1] = rng.integers(0, 5, nvox)
    x0[::w * h, 2] = 1
    return W.make_problem(W.model_notch_paper(), lattice=lattice, nx=nx, ny=ny, mesh_w=w, mesh_h=h,
                          rates=[100.0, 64.0, 25.0, 1.0, 1.0], trans_rate=2.0,
                          diffusion=[16.0, 16.0, 0.0, 0.0], init_counts=x0, seed=seed, dt=0.05,
                          n_steps=n_steps)


def _whole(p, n_steps, chunks=None, trace=True, allow_flags=False):
    from paper_1806_10889_amd import tissue as T
    t = T.Tissue(p, trace_steps=n_steps if trace else 0)
    assert t.runs_whole(), "the whole-run kernel should take this tissue"
    for c in (chunks or [n_steps]):
        t.step(p["dt"], c)
    out = dict(counts=t.read_counts(allow_flags=allow_flags), stats=t.stats())
    if trace:
        out["trace"] = t.trace(int(p.get("start_step", 0)), n_steps)
    t.close()
    return out


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_config1_full_horizon(oracle_lib, scheme):
    """The 16 well-mixed cells of the small workload over their whole
    horizon (100 steps, one launch), trans signalling over four colour
    classes of edges that share their cells' single voxel."""
    p = dict(W.config1(), scheme=scheme)
    o = oracle_lib.run(p, p["dt"], 100, trace=True)
    assert_same(_whole(p, 100), o)


@pytest.mark.parametrize("lattice", [0, 1])
@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_first_order_overlapping_faces_across_launches(oracle_lib, lattice, scheme):
    """36 cells of 2 x 2 voxels (face groups that share their corner
    voxels: several S passes), first-order signalling with diffusion in the
    cells, 160 steps in calls of 3, 150 and 7 (the middle call spans two
    launches of at most 100 steps)."""
    p = dict(_cells(31 + lattice, lattice, 160, 2, 2), scheme=scheme)
    o = oracle_lib.run(p, p["dt"], 160, trace=True)
    assert_same(_whole(p, 160, chunks=[3, 150, 7]), o)
    # the step-by-step launches give the same bits
    assert_same(gpu_run(p, 160, trace=True, chunks=[3, 150, 7]), o)


def test_resumed_run(oracle_lib):
    """A run resumed at step 1000 (the counters' step field) of a tissue
    whose square lattice gives every cell one voxel in four face groups."""
    p = dict(W.config1(seed=8), start_step=1000)
    o = oracle_lib.run(p, p["dt"], 40, trace=True)
    assert_same(_whole(p, 40), o)


def test_batches_of_small_tissues(oracle_lib):
    """A batch of one small tissue runs whole; a batch of two runs step by
    step (two chi items); both as each tissue runs alone."""
    from paper_1806_10889_amd import tissue as T
    for n in (1, 2):
        probs = [dict(W.config1(seed=s), sim_id=s) for s in range(3, 3 + n)]
        ts = [T.Tissue(p) for p in probs]
        b = T.Batch(ts)
        assert b.runs_whole() == (n == 1)
        b.step(probs[0]["dt"], 60)
        b.sync()
        for p, t in zip(probs, ts):
            o = oracle_lib.run(p, p["dt"], 60)
            st = t.stats()
            assert np.array_equal(t.read_counts(), o.counts)
            assert (st["chi_events"], st["s_events"], st["draws"]) == (o.chi_events, o.s_events, o.draws)
        b.close()
        for t in ts:
            t.close()


def test_flags_in_the_whole_run(oracle_lib):
    """A count crossing 2^26 and a cell-step at the event cap flag the
    tissue as in the step-by-step launches, with the oracle's counts."""
    from paper_1806_10889_amd import tissue as T
    net = W._net(["A", "B"], [("make", [], {"A": 1}), ("turn", ["A"], {"B": 1})], None)
    x0 = np.zeros((4, 2), np.int32)
    x0[0, 0] = (1 << 26) - 5
    p = W.make_problem(net, lattice=0, nx=2, ny=2, mesh_w=1, mesh_h=1, rates=[50.0, 1e-9],
                       trans_rate=0.0, diffusion=[0.0, 0.0], init_counts=x0, seed=17, dt=1.0,
                       n_steps=2)
    o = oracle_lib.run(p, 1.0, 2)
    assert o.overflow
    assert_same(_whole(p, 2, trace=False, allow_flags=True), o, trace=False)
    q = W.make_problem(net, lattice=0, nx=2, ny=2, mesh_w=2, mesh_h=2, rates=[20.0, 0.5],
                       trans_rate=0.0, diffusion=[1.0, 0.5], init_counts=np.zeros((16, 2), np.int32),
                       seed=23, dt=1.0, n_steps=2, event_cap=50)
    o = oracle_lib.run(q, 1.0, 2)
    assert o.capped
    g = _whole(q, 2, trace=False, allow_flags=True)
    assert_same(g, o, trace=False)
    t = T.Tissue(q)
    t.step(1.0, 2)
    with pytest.raises(T.TissueError) as ei:
        t.read_counts()
    assert ei.value.code == T.ELIMIT
    t.close()


def test_when_the_whole_run_applies():
    """It takes a tissue whose chi operator is one item of the lane layout
    with a compiled network; not one of several leaf classes, not more than
    64 cells, not cells of more than 8 voxels, not a generic network, and
    not when switched off."""
    from paper_1806_10889_amd import tissue as T
    t = T.Tissue(W.config1())
    assert t.runs_whole()
    t.set_whole_run(False)
    assert not t.runs_whole()
    t.set_whole_run(True)
    t.set_chi_mode(1)  # rows
    assert not t.runs_whole()
    t.close()
    h = np.tile([1, 2], 8)
    mixed = W.make_problem(W.model_notch_paper(), lattice=0, nx=4, ny=4, mesh_w=1, mesh_h=h,
                           rates=[1.0] * 5, trans_rate=1.0, diffusion=[1.0, 1.0, 0.0, 0.0],
                           init_counts=np.ones((int(h.sum()), 4), np.int32), seed=5, dt=0.1,
                           n_steps=2)
    t = T.Tissue(mixed)  # classes of 1 and 2 leaves: two chi items
    assert not t.runs_whole()
    t.close()
    big = W.birth_death(1.0, 0.1, 5, nx=9, ny=8)  # 72 cells: two items
    t = T.Tissue(big)
    assert not t.runs_whole()
    t.close()
    t = T.Tissue(W.config2(side=4, n_steps=2))  # 4x4-voxel cells: rows
    assert not t.runs_whole()
    t.close()
    t = T.Tissue(W.config1(), jit=False)
    assert not t.runs_whole()
    t.close()
