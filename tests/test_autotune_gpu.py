"""Autotuner: the chosen launch shape is applied and leaves the bits alone;
a second call with the same workload shape hits the cache."""
import numpy as np
import pytest

from paper_1806_10889_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_keeps_bits_and_caches(oracle_lib, tmp_path, monkeypatch):
    from paper_1806_10889_amd import autotune, tissue as T
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    p = W.config2(side=12, n_steps=6)
    t = T.Tissue(p)
    r1 = autotune.tune([p], p["dt"], steps=6, reps=1, target=t)
    assert not r1["cached"] and r1["candidates"] >= 8
    t.step(p["dt"], 6)
    o = oracle_lib.run(p, p["dt"], 6)
    assert np.array_equal(t.read_counts(), o.counts)
    q = W.config2(side=12, n_steps=6, seed=99)  # same shape, other draws
    r2 = autotune.tune([q], q["dt"], steps=6, reps=1)
    assert r2["cached"] and r2["config"] == r1["config"]
