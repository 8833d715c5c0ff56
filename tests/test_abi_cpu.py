"""The C-ABI library loads and exports every declared entry point, and its
host-side validation rejects bad descriptors (CPU only: no compute call)."""
import os
import re

import numpy as np
import pytest

from paper_1806_10889_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tissue.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tissue_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1806_10889_amd import tissue as T
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(T.lib, n), n
    assert sorted(T.EXPORTS) == names


def bad_of(p, mut):
    from paper_1806_10889_amd import tissue as T
    q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    mut(q)
    assert T.required_bytes(q) == 0, T.lib.tissue_last_error()
    return T.lib.tissue_last_error().decode()


def test_required_bytes_and_validation():
    from paper_1806_10889_amd import tissue as T
    p = W.config2(side=8)
    assert T.required_bytes(p) > W.n_voxels(p) * 5 * 4 * 2
    assert T.required_bytes(W.config1()) > 0
    assert T.required_bytes(p, trace_steps=5) > T.required_bytes(p)

    def bad(mut):
        q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
        mut(q)
        assert T.required_bytes(q) == 0, T.lib.tissue_last_error()
        return T.lib.tissue_last_error().decode()

    assert "rates" in bad(lambda q: q["rates"].__setitem__(0, -1.0))
    assert "rates" in bad(lambda q: q["rates"].__setitem__(0, float("nan")))
    assert "diffusion" in bad(lambda q: q["diffusion"].__setitem__(0, float("inf")))
    assert "init_counts" in bad(lambda q: q["init_counts"].__setitem__((0, 0), -1))
    assert "init_counts" in bad(lambda q: q["init_counts"].__setitem__((0, 0), 1 << 26))
    assert "mesh" in bad(lambda q: q["mesh_w"].__setitem__(0, 9))
    assert "mesh" in bad(lambda q: q["mesh_h"].__setitem__(3, 0))
    assert "sim_id" in bad(lambda q: q.__setitem__("sim_id", 1 << 30))
    assert "distinct" in bad(lambda q: q.__setitem__("trans_d", q["trans_n"]))
    assert "lattice" in bad(lambda q: q.__setitem__("lattice", 2))

    def consume_unsupplied(q):
        q["stoich"] = q["stoich"].copy()
        q["stoich"][0, 1] = -1  # 0 -> N would also remove a D it does not have
    assert "consumes" in bad(consume_unsupplied)

    def reactant_range(q):
        q["reactants"] = q["reactants"].copy()
        q["reactants"][1, 0] = 7
    assert "reactant" in bad(reactant_range)

    # flags: unknown bits are refused; the Strang flag is accepted and does
    # not change the layout
    h = T._DescHolder(p)
    h.desc.flags = 16
    assert T.lib.tissue_required_bytes(T.C.byref(h.desc)) == 0
    assert "flags" in T.lib.tissue_last_error().decode()
    # first-order signalling: trans_n unused, trans_d and trans_i distinct
    n = W.config_notch(side=4, n_steps=1)
    assert T._DescHolder(n).desc.flags & T.FLAG_SIGNAL_FIRST_ORDER
    assert n["trans_n"] == -1 and T.required_bytes(n) > 0
    assert "distinct" in bad_of(n, lambda q: q.__setitem__("trans_i", q["trans_d"]))
    try:
        T._DescHolder(dict(n, signal="second_order"))
    except ValueError as e:
        assert "signal" in str(e)
    else:
        raise AssertionError("expected a ValueError")
    q = dict(p)
    q["scheme"] = "strang"
    assert T.required_bytes(q) == T.required_bytes(p)
    h = T._DescHolder(q)
    assert h.desc.flags & T.FLAG_STRANG
    try:
        T._DescHolder(dict(p, scheme="leapfrog"))
    except ValueError as e:
        assert "scheme" in str(e)
    else:
        raise AssertionError("expected a ValueError")


def test_error_strings():
    from paper_1806_10889_amd import tissue as T
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert T.lib.tissue_strerror(code)
    assert T.lib.tissue_strerror(-99) == b"unknown error"


@pytest.mark.parametrize("model", ["nd5", "nd4", "bd", "dimer", "diff", "tr"])
def test_network_kernels_compile(model):
    """The chi kernels compiled per network (hipRTC, gfx950) build for every
    test network; no device needed."""
    from paper_1806_10889_amd import tissue as T
    p = W.random_problem(1, lattice=0, nx=2, ny=2, model=model, mesh=(2, 2))
    T.network_check(p)


def test_per_cell_model_validation():
    """Per-cell models: the extra networks obey the same table rules (the
    message names the model), cell_model entries stay within n_models, at
    most 7 extra networks; each extra network adds its table to the buffer."""
    from paper_1806_10889_amd import tissue as T
    p = W.config_multifidelity(side=6, rim=1, n_steps=2)
    base = W.config_notch(side=6, n_steps=2)
    assert T.required_bytes(p) > 0
    one = dict(reactants=p["reactants"], stoich=p["stoich"], rates=p["rates"],
               diffusion=p["diffusion"])
    assert "cell_model" in bad_of(p, lambda q: q["cell_model"].__setitem__(0, 2))
    assert "n_models" in bad_of(p, lambda q: q.__setitem__("models", [one] * 8))

    def bad_model(q):
        m = dict(q["models"][0])
        r = np.array(m["reactants"]).copy()
        r[1, 0] = 9
        m["reactants"] = r
        q["models"] = [m]
    assert "model 1" in bad_of(p, bad_model)

    def neg_rate(q):
        m = dict(q["models"][0])
        m["rates"] = np.array(m["rates"]) * -1.0
        q["models"] = [m]
    assert "model 1" in bad_of(p, neg_rate)
    # a model's table in the device buffer (aligned, so at least 256 bytes more)
    q = W.with_models(base, [one], np.zeros(36, np.int32))
    assert T.required_bytes(q) >= T.required_bytes(base) + 256


def test_per_cell_models_compile():
    """Every network of a multi-fidelity tissue gets compiled chi kernels."""
    from paper_1806_10889_amd import tissue as T
    T.network_check(W.config_multifidelity(side=4, rim=1, n_steps=2))


def test_per_cell_signal_rate_validation():
    """A network's first-order signalling rate is checked like trans_rate;
    under the second-order reaction it has to equal trans_rate."""
    p = W.config_multifidelity(side=5, rim=1, n_steps=2)

    def rate(v):
        def mut(q):
            q["models"] = [dict(q["models"][0], signal_rate=v)]
        return mut
    assert "signal_rate" in bad_of(p, rate(-1.0))
    assert "signal_rate" in bad_of(p, rate(float("nan")))
    q = W.config2(side=5, n_steps=2)
    one = dict(reactants=q["reactants"], stoich=q["stoich"], rates=q["rates"],
               diffusion=q["diffusion"])
    q2 = W.with_models(q, [dict(one, signal_rate=q["trans_rate"] * 2)], np.arange(25) % 2)
    assert "second-order" in bad_of(q2, lambda r: None)
    from paper_1806_10889_amd import tissue as T
    assert T.required_bytes(W.with_models(q, [one], np.arange(25) % 2)) > 0
