"""GPU parity of per-cell models: cells of one tissue running different
networks (the paper's Discussion: detailed modules where cells signal,
coarser ones where little happens), through the C-ABI against the oracle,
bit for bit on counts, traces and totals."""
import numpy as np
import pytest

from gpu_helpers import assert_same, gpu_run, notch_uneven
from paper_1806_10889_amd import workloads as W

pytestmark = pytest.mark.gpu

MODES = [0, 1, 2, 3, 4]


def _nd5_mixed(seed, *, uneven=True, lattice=1, nx=9, ny=7, n_steps=5):
    """An nd5 tissue whose cells run one of four networks: the tissue's own,
    the same structure with other rates, every other reaction with one
    diffusing species, and pure diffusion (no reactions)."""
    p = W.random_problem(seed, lattice=lattice, nx=nx, ny=ny, model="nd5", uneven=uneven,
                         mesh=None if uneven else (4, 4), dt=0.05, n_steps=n_steps)
    rng = np.random.default_rng(seed)
    re, st = np.asarray(p["reactants"]).reshape(-1, 2), np.asarray(p["stoich"]).reshape(-1, 5)
    same = dict(reactants=re, stoich=st, rates=10.0 ** rng.uniform(-2, 1, re.shape[0]),
                diffusion=p["diffusion"])
    half = dict(reactants=re[::2], stoich=st[::2], rates=10.0 ** rng.uniform(-2, 1, re[::2].shape[0]),
                diffusion=[2.0, 0.0, 0.0, 0.0, 0.0])
    none = dict(reactants=np.zeros((0, 2), np.int32), stoich=np.zeros((0, 5), np.int32), rates=[],
                diffusion=[0.5, 1.5, 0.0, 3.0, 0.0])
    cm = rng.integers(0, 4, nx * ny)
    return W.with_models(p, [same, half, none], cm)


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mode", MODES)
def test_multi_fidelity_notch(oracle_lib, mode, jit):
    p = W.config_multifidelity(side=8, rim=2, n_steps=8)
    o = oracle_lib.run(p, p["dt"], 8, trace=True)
    assert o.s_events > 0 and o.chi_events > 1000
    assert_same(gpu_run(p, 8, trace=True, chi_mode=mode, jit=jit), o)


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mode", MODES)
def test_four_networks_uneven_meshes(oracle_lib, mode, jit):
    p = _nd5_mixed(61)
    o = oracle_lib.run(p, p["dt"], 5, trace=True)
    assert o.chi_events > 10000 and o.s_events > 0
    assert_same(gpu_run(p, 5, trace=True, chi_mode=mode, jit=jit), o)


@pytest.mark.parametrize("persistent", [False, True])
def test_four_networks_regrouped_by_load(oracle_lib, persistent):
    """The compact layout with the regroup pass forced on: each (class,
    network) launch reorders its own cells by load between steps; same
    bits."""
    p = _nd5_mixed(63, n_steps=6)
    o = oracle_lib.run(p, p["dt"], 6, trace=True)
    assert_same(gpu_run(p, 6, trace=True, chi_mode=3, regroup=1, persistent=persistent,
                        graph_chunk=2), o)


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_networks_in_forked_graphs_and_redo(oracle_lib, scheme):
    """One workgroup per item and captured graphs (the (class, network)
    launches as parallel branches), compact layout with wide counts in cells
    of several networks: same bits."""
    p = _nd5_mixed(62, uneven=False, n_steps=4)
    p["scheme"] = scheme
    x = p["init_counts"].reshape(63, 16, 5)
    for m in range(4):
        x[np.flatnonzero(p["cell_model"] == m)[0], 3, 0] = 65535
    o = oracle_lib.run(p, p["dt"], 4, trace=True)
    for mode in (3, 0, 1):
        assert_same(gpu_run(p, 4, trace=True, persistent=False, graph_chunk=2, chi_mode=mode), o)


def test_every_cell_on_an_extra_network_and_unused_networks(oracle_lib):
    """No cell on the tissue's own network, one extra network unused."""
    p = _nd5_mixed(63, n_steps=4)
    p["cell_model"][:] = np.where(np.arange(63) % 2 == 0, 1, 3)
    o = oracle_lib.run(p, p["dt"], 4, trace=True)
    assert_same(gpu_run(p, 4, trace=True), o)


def test_model_tissues_share_a_batch(oracle_lib):
    from paper_1806_10889_amd import tissue as T
    probs = [_nd5_mixed(64, n_steps=5), W.config2(side=6, n_steps=5),
             W.config_multifidelity(side=6, rim=1, n_steps=5), _nd5_mixed(65, lattice=0, n_steps=5)]
    for i, p in enumerate(probs):
        p["dt"] = 0.05
        p["sim_id"] = i
    ts = [T.Tissue(p, jit=(i != 3)) for i, p in enumerate(probs)]
    b = T.Batch(ts)
    b.step(0.05, 3)
    b.set_chi_mode(3)
    b.step(0.05, 2)
    b.sync()
    for p, t in zip(probs, ts):
        o = oracle_lib.run(p, 0.05, 5)
        assert_same(dict(counts=t.read_counts(), stats=t.stats()), o, trace=False)
    b.close()
    for t in ts:
        t.close()


@pytest.mark.parametrize("scheme", ["lie", "strang"])
@pytest.mark.parametrize("lattice", [0, 1])
def test_first_order_rates_per_network(oracle_lib, lattice, scheme):
    """The paper's network on uneven meshes with three networks whose cells
    signal at different first-order rates (one of them zero): each side of
    an edge at its own cell's rate; every chi mode."""
    p = notch_uneven(70 + lattice, lattice, scheme)
    base = dict(reactants=p["reactants"], stoich=p["stoich"], rates=p["rates"],
                diffusion=p["diffusion"])
    rng = np.random.default_rng(lattice)
    p = W.with_models(p, [dict(base, signal_rate=7.5),
                          dict(base, rates=[60.0, 10.0, 5.0, 2.0, 0.5], signal_rate=0.0)],
                      rng.integers(0, 3, 30))
    o = oracle_lib.run(p, p["dt"], 5, trace=True)
    assert o.s_events > 100
    for mode in MODES:
        assert_same(gpu_run(p, 5, trace=True, chi_mode=mode), o)
