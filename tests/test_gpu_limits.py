"""The descriptor's table maxima on the GPU: a network of 8 species (the
packed net changes of species 4..7 in the second word) and 16 reactions of
every order (productions, conversions, bindings and dimerisations
x(x-1)/2), every species diffusing (24 channel slots per voxel), with the
trans reaction between three of the species; bit-exact against the oracle
in every chi layout, compiled and generic networks, cells of 2x2, 4x4 and
8x8 voxels, Lie and Strang splitting, and through the whole-run kernel."""
import numpy as np
import pytest

from gpu_helpers import assert_same, gpu_run
from paper_1806_10889_amd import workloads as W

pytestmark = pytest.mark.gpu

MODES = [0, 1, 3, 4]


def max_network(seed):
    rng = np.random.default_rng(seed)
    sp = [f"S{k}" for k in range(8)]
    rx = []
    for r in range(16):
        a, b, c = (sp[int(x)] for x in rng.choice(8, size=3, replace=False))
        kind = r % 4
        if kind == 0:
            rx.append((f"make{r}", [], {c: 1}))
        elif kind == 1:
            rx.append((f"conv{r}", [a], {a: -1, c: 1}))
        elif kind == 2:
            rx.append((f"bind{r}", [a, b], {a: -1, b: -1, c: 1}))
        else:
            rx.append((f"dimer{r}", [a, a], {a: -2, c: 1}))
    return W._net(sp, rx, (sp[0], sp[1], sp[2]))


def max_problem(seed, mesh, nx=4, ny=3, n_steps=4, scheme="lie"):
    m = max_network(seed)
    assert m["n_species"] == 8 and m["n_reactions"] == 16
    rng = np.random.default_rng(seed + 100)
    w, h = mesh
    p = W.make_problem(m, lattice=1, nx=nx, ny=ny, mesh_w=w, mesh_h=h,
                       rates=10.0 ** rng.uniform(-2, 0, 16), trans_rate=0.5,
                       diffusion=np.full(8, 0.8),
                       init_counts=rng.integers(0, 30, size=(nx * ny * w * h, 8)),
                       seed=seed, dt=0.05, n_steps=n_steps)
    p["scheme"] = scheme
    return p


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("mesh", [(2, 2), (4, 4), (8, 8)])
def test_maximal_network_every_layout(oracle_lib, mesh, mode, jit):
    p = max_problem(61 + mesh[0], mesh)
    o = oracle_lib.run(p, p["dt"], 4, trace=True)
    assert_same(gpu_run(p, 4, trace=True, chi_mode=mode, jit=jit), o)


@pytest.mark.parametrize("mode", [1, 3])
def test_maximal_network_strang(oracle_lib, mode):
    p = max_problem(71, (4, 4), scheme="strang")
    o = oracle_lib.run(p, p["dt"], 4, trace=True)
    assert_same(gpu_run(p, 4, trace=True, chi_mode=mode), o)


def test_maximal_network_whole_run(oracle_lib):
    from paper_1806_10889_amd import tissue as T
    p = max_problem(81, (2, 2), n_steps=30)
    o = oracle_lib.run(p, p["dt"], 30, trace=True)
    t = T.Tissue(p, trace_steps=30)
    assert t.runs_whole()
    t.step(p["dt"], 30)
    g = dict(counts=t.read_counts(), stats=t.stats(), trace=t.trace(0, 30))
    t.close()
    assert_same(g, o)
