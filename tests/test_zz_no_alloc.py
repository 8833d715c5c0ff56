"""The no-allocation batch step (tissue_batch_step_static) against the batch
step with a caller's workspace (tissue_batch_step): the same tissues, the
same steps, bit-identical counts and totals -- on two calls in a row, the
second with a smaller batch, so that it runs on what the first left in the
static workspace -- and a batch too large for the workspace is refused
before anything is enqueued."""
import numpy as np
import pytest

from paper_1806_10889_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problems():
    return [
        W.random_problem(180, lattice=1, nx=9, ny=9, model="nd5", mesh=(4, 4), dt=0.05, sim_id=3),
        W.random_problem(181, lattice=1, nx=5, ny=7, model="nd5", uneven=True, dt=0.05, sim_id=4),
        W.random_problem(182, lattice=0, nx=6, ny=4, model="nd4", mesh=(1, 1), dt=0.05, sim_id=5),
        W.random_problem(183, lattice=1, nx=40, ny=40, model="nd5", mesh=(4, 4), dt=0.05, sim_id=6),
        W.random_problem(184, lattice=0, nx=3, ny=3, model="nd5", mesh=(8, 8), dt=0.05, sim_id=7),
    ]


def _same(a, b):
    assert np.array_equal(a.read_counts(), b.read_counts())
    sa, sb = a.stats(), b.stats()
    for k in ("chi_events", "s_events", "draws", "steps_done"):
        assert sa[k] == sb[k], k


def test_static_batch_step_equals_batch_step():
    from paper_1806_10889_amd import tissue as T
    probs = _problems()
    probs[1]["start_step"] = 11
    # the wide-count redo of the compact layout in the 40x40 member
    probs[3]["init_counts"].reshape(1600, 16, 5)[[7, 900], 3, 0] = 65534
    ref = [T.Tissue(p) for p in probs]
    got = [T.Tissue(p) for p in probs]
    b = T.Batch(ref)
    b.step(0.05, 4)
    b.sync()
    T.batch_step_static(got, 0.05, 4)
    for a, g in zip(ref, got):
        _same(a, g)
    b.close()
    # second call, smaller: three of the tissues, further on
    sub = [0, 2, 4]
    b2 = T.Batch([ref[i] for i in sub])
    b2.step(0.05, 3)
    b2.sync()
    T.batch_step_static([got[i] for i in sub], 0.05, 3)
    for i in sub:
        _same(ref[i], got[i])
    b2.close()
    for t in ref + got:
        t.close()


def test_static_batch_step_refuses_what_does_not_fit():
    from paper_1806_10889_amd import tissue as T
    p = W.birth_death(1.0, 0.1, 3, nx=1500, ny=1500, dt=0.1)  # 2.25 M cells: > 32 MiB of work lists
    t = T.Tissue(p)
    with pytest.raises(T.TissueError) as ei:
        T.batch_step_static([t], 0.1, 1)
    assert ei.value.code == T.ENOMEM and "workspace" in str(ei.value)
    with pytest.raises(T.TissueError) as ei:
        T.batch_step_static([t, t], 0.1, 1)
    assert ei.value.code == T.EINVAL
    assert t.stats()["steps_done"] == 0 and t.stats()["draws"] == 0
    t.close()
