"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): oracle.c built with both, every run path exercised in a child
process (uneven meshes on both lattices with overlapping faces, the
paper's first-order signalling, Strang splitting, per-cell networks, a
capped unit-step), any report aborting it, and the results equal to those
of the ordinary build."""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[2])
import oracle
from paper_1806_10889_amd import workloads as W
from gpu_helpers import notch_uneven
out = []
for p in cases():
    r = oracle.run(p, p["dt"], p["n_steps"], trace=True, threads=1)
    out.append(np.concatenate([r.counts.astype(np.int64), [r.chi_events, r.s_events, r.draws]]))
np.save(sys.argv[3], np.concatenate(out))
"""

CASES = r"""
def cases():
    ps = [W.random_problem(5, lattice=0, nx=5, ny=4, model="nd5", uneven=True, n_steps=3),
          W.random_problem(6, lattice=1, nx=4, ny=5, model="nd4", uneven=True, n_steps=3),
          notch_uneven(7, 1, "strang", n_steps=3),
          W.config_multifidelity(side=6, rim=1, dt=0.1, n_steps=3)]
    capped = W.random_problem(8, lattice=1, nx=3, ny=3, model="bd", mesh=(2, 2), n_steps=2)
    capped["event_cap"] = 50
    return ps + [capped]
"""


def _libasan():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(_libasan() is None, reason="gcc has no AddressSanitizer runtime here")
def test_oracle_clean_under_asan_and_ubsan():
    import oracle
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liboracle_san.so")
        subprocess.check_call(["gcc", *[f for f in oracle.CFLAGS if f != "-O2"], "-O1", "-g",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               "-fno-omit-frame-pointer", "-o", lib, oracle._SRC, "-lm"])
        script = os.path.join(d, "child.py")
        with open(script, "w") as f:
            f.write(CHILD.replace("for p in cases():", CASES + "\nfor p in cases():"))
        env = dict(os.environ, ORACLE_LIBRARY=lib, LD_PRELOAD=_libasan(),
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="1")
        res = subprocess.run([sys.executable, script, ROOT, os.path.join(ROOT, "tests"),
                              os.path.join(d, "san.npy")], env=env, capture_output=True, text=True,
                             timeout=600)
        assert res.returncode == 0, res.stderr[-4000:]
        got = np.load(os.path.join(d, "san.npy"))
    # the same cases through the ordinary build, in this process
    ns = {}
    exec("from paper_1806_10889_amd import workloads as W\nfrom gpu_helpers import notch_uneven\n" + CASES, ns)
    ref = []
    for p in ns["cases"]():
        r = oracle.run(p, p["dt"], p["n_steps"], trace=True, threads=1)
        ref.append(np.concatenate([r.counts.astype(np.int64), [r.chi_events, r.s_events, r.draws]]))
    assert np.array_equal(got, np.concatenate(ref))
