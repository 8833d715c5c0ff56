"""Pins for the oracle's random stream and log (CPU only).

Philox4x32-10 (Salmon et al., SC'11): a generic Philox-4xW written in
Python is checked against numpy's Philox4x64-10 (an independent
implementation of the same family); the same generic code at W=32 with the
paper's 4x32 constants must equal the oracle; the Weyl constants are
recomputed from their definition; and the oracle reproduces the published
known-answer vectors.  plog is checked against mpmath to 2 ulp.
"""
import math
import os

import numpy as np
import pytest

import refmath

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_generic_philox_matches_numpy_4x64():
    rng = np.random.default_rng(0)
    for _ in range(50):
        key = [int(v) for v in rng.integers(0, 2 ** 63, size=2, dtype=np.uint64)]
        c0 = int(rng.integers(0, 2 ** 62))
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array([c0, 0, 0, 0], dtype=np.uint64))
        raw = [int(v) for v in bg.random_raw(8)]
        # numpy advances the counter before generating each block
        exp = refmath.philox4([c0 + 1, 0, 0, 0], key, **refmath.PHILOX4x64) + \
            refmath.philox4([c0 + 2, 0, 0, 0], key, **refmath.PHILOX4x64)
        assert raw == exp


def test_weyl_constants_from_definition():
    import mpmath
    mpmath.mp.prec = 200
    phi_m1 = (mpmath.sqrt(5) - 1) / 2
    sqrt3_m1 = mpmath.sqrt(3) - 1
    assert int(mpmath.floor(phi_m1 * 2 ** 32)) == refmath.PHILOX4x32["W0"]
    assert int(mpmath.floor(sqrt3_m1 * 2 ** 32)) == refmath.PHILOX4x32["W1"]
    assert int(mpmath.floor(phi_m1 * 2 ** 64)) == refmath.PHILOX4x64["W0"]
    assert int(mpmath.floor(sqrt3_m1 * 2 ** 64)) == refmath.PHILOX4x64["W1"]


def test_oracle_philox_known_answers(oracle_lib):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle_lib.philox(v[0:4], v[4:6]) == tuple(v[6:10])
        assert tuple(refmath.philox4x32(v[0:4], v[4:6])) == tuple(v[6:10])


def test_oracle_philox_matches_generic_4x32(oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(300):
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)]
        assert oracle_lib.philox(ctr, key) == tuple(refmath.philox4x32(ctr, key))


def test_uniform_edges(oracle_lib):
    u1, u2 = oracle_lib.uniforms([0, 0, 0, 0])
    assert u1 == 2.0 ** -53 and u2 == 0.0
    u1, u2 = oracle_lib.uniforms([0xFFFFFFFF] * 4)
    assert u1 == 1.0 and u2 == 1.0 - 2.0 ** -53
    # low 11 bits are dropped
    u1, u2 = oracle_lib.uniforms([0, 0x7FF, 0, 0x7FF])
    assert u1 == 2.0 ** -53 and u2 == 0.0
    u1, u2 = oracle_lib.uniforms([0, 0x800, 0, 0x800])
    assert u1 == 2.0 * 2.0 ** -53 and u2 == 2.0 ** -53
    rng = np.random.default_rng(2)
    for _ in range(200):
        w = [int(v) for v in rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        assert oracle_lib.uniforms(w) == refmath.uniforms(w)


def _ulp_err(x):
    import mpmath
    got = oracle_lib_plog(x)
    exact = mpmath.log(mpmath.mpf(x))
    if exact == 0:
        return 0.0 if got == 0.0 else float("inf")
    ulp = math.ulp(float(exact))
    return float(abs(mpmath.mpf(got) - exact) / ulp)


oracle_lib_plog = None


def test_plog_accuracy_vs_mpmath(oracle_lib):
    import mpmath
    global oracle_lib_plog
    oracle_lib_plog = oracle_lib.plog
    mpmath.mp.prec = 120
    assert oracle_lib.plog(1.0) == 0.0
    worst = 0.0
    pts = [2.0 ** -k for k in range(0, 54)]
    pts += [math.nextafter(2.0 ** -k, 0.0) for k in range(0, 53)]
    pts += [math.sqrt(2.0) * 2.0 ** -k for k in range(1, 52)]
    rng = np.random.default_rng(3)
    # the uniforms actually fed to plog: (m + 1) 2^-53
    ms = rng.integers(0, 2 ** 53, size=20000, dtype=np.uint64)
    pts += [float(int(m) + 1) * 2.0 ** -53 for m in ms]
    pts += list(rng.uniform(0.5, 1.0, size=5000))
    pts += list(np.exp(rng.uniform(-36.0, 0.0, size=5000)))
    for x in pts:
        worst = max(worst, _ulp_err(float(x)))
    assert worst <= 2.0, worst


def test_plog_python_restatement_matches_oracle(oracle_lib):
    rng = np.random.default_rng(4)
    for x in list(rng.uniform(2.0 ** -53, 1.0, size=300)) + [1.0, 0.5, 2.0 ** -53]:
        assert refmath.plog_py(float(x)) == oracle_lib.plog(float(x))
