"""Pins for the oracle's simulation (CPU only).

The oracle's trajectories are one realisation of the split Markov process,
so its *law* is pinned against what the mathematics fixes:

* a textbook direct method (Gillespie), written independently, on
  well-mixed cells: bit-equal trajectories on the same random stream;
* birth-death: transient law Bin(x0, e^{-gamma t}) + Poisson(k/gamma (1 -
  e^{-gamma t})) and stationary law Poisson(k/gamma);
* order-2 same-species propensity x(x-1)/2: CME solved by expm;
* diffusion: one molecule's law is e^{tQ}, n molecules are multinomial;
* the splitting scheme itself (chi over dt, then S over dt): brute-force CME
  of the split process by expm on tiny closed tissues, which the reversed
  order fails; and its convergence to the unsplit CME as dt -> 0;
* conservation invariants of the Notch networks; chunking/resume identity.
"""
import math

import numpy as np
import pytest
from scipy import linalg, stats

import refmath
from paper_1806_10889_amd import workloads as W
from splitlaw import split_law as _split_law, two_cell_nd5 as _two_cell_nd5


def _sample_bd(oracle_lib, k, gamma, x0, dt, n_steps, side=100, seed=11):
    p = W.birth_death(k, gamma, x0, nx=side, ny=side, dt=dt, n_steps=n_steps, seed=seed)
    r = oracle_lib.run(p, dt, n_steps)
    return r.counts.astype(np.int64)


def test_textbook_direct_method_bit_equal_config1(oracle_lib):
    p = W.config1()
    want = refmath.textbook_v1(p, p["n_steps"])
    got = oracle_lib.run(p, p["dt"], p["n_steps"]).counts
    assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", [21, 22])
def test_textbook_direct_method_bit_equal_busy(oracle_lib, seed):
    p = W.random_problem(seed, lattice=0, nx=3, ny=3, model="nd4", mesh=(1, 1),
                         dt=0.1, n_steps=8, rate_lo=-1.0, rate_hi=1.0, count_hi=30)
    r = oracle_lib.run(p, p["dt"], p["n_steps"])
    assert r.chi_events > 200 and r.s_events > 10
    assert np.array_equal(r.counts, refmath.textbook_v1(p, p["n_steps"]))


def test_birth_death_transient_law(oracle_lib):
    k, gamma, x0, dt, n = 5.0, 0.5, 20, 0.1, 20
    x = _sample_bd(oracle_lib, k, gamma, x0, dt, n)
    t = dt * n
    q = math.exp(-gamma * t)
    mean = x0 * q + (k / gamma) * (1 - q)
    var = x0 * q * (1 - q) + (k / gamma) * (1 - q)
    N = x.size
    assert abs(x.mean() - mean) < 3 * math.sqrt(var / N)
    # variance: SE from the fourth central moment of the exact law
    support = np.arange(0, 120)
    pmf = np.convolve(stats.binom.pmf(np.arange(0, x0 + 1), x0, q),
                      stats.poisson.pmf(support, (k / gamma) * (1 - q)))[:120]
    m4 = float(np.sum(pmf * (np.arange(120) - mean) ** 4))
    se_var = math.sqrt((m4 - var ** 2) / N)
    assert abs(x.var() - var) < 3 * se_var
    obs = np.bincount(x, minlength=120)[:120]
    pval, _, _ = refmath.chisquare_pvalue(obs, pmf * N)
    assert pval > 0.01
    # KS after the randomised probability-integral transform, which maps a
    # sample of a discrete law to an exact U(0,1) sample
    assert refmath.discrete_ks_pvalue(x, pmf) > 0.01


def test_birth_death_stationary_poisson(oracle_lib):
    k, gamma = 8.0, 1.0
    x = _sample_bd(oracle_lib, k, gamma, 0, 0.5, 40, seed=13)  # gamma T = 20
    lam = k / gamma
    N = x.size
    assert abs(x.mean() - lam) < 3 * math.sqrt(lam / N)
    se_var = math.sqrt((lam + 3 * lam ** 2 - lam ** 2) / N)  # Poisson mu4 = lam + 3 lam^2
    assert abs(x.var() - lam) < 3 * se_var
    obs = np.bincount(x, minlength=60)[:60]
    pmf = stats.poisson.pmf(np.arange(60), lam)
    pval, _, _ = refmath.chisquare_pvalue(obs, pmf * N)
    assert pval > 0.01
    assert refmath.discrete_ks_pvalue(x, pmf) > 0.01


def test_dimerisation_cme(oracle_lib):
    """0 -> X (k), X + X -> 0 (c x(x-1)/2): law at T by expm of the CME."""
    k, c, x0, dt, n = 6.0, 0.4, 10, 0.1, 10
    m = W.model_dimer()
    side = 100
    p = W.make_problem(m, lattice=0, nx=side, ny=side, mesh_w=1, mesh_h=1, rates=[k, c],
                       trans_rate=0.0, diffusion=0.0,
                       init_counts=np.full((side * side, 1), x0, np.int32), seed=17,
                       dt=dt, n_steps=n)
    x = oracle_lib.run(p, dt, n).counts.astype(np.int64)
    top = 80

    def tr(s):
        (v,) = s
        out = []
        if v < top:
            out.append((k, (v + 1,)))
        if v >= 2:
            out.append((c * v * (v - 1) / 2, (v - 2,)))
        return out
    states, index = refmath.enumerate_states((x0,), tr)
    Q = refmath.generator(states, index, tr)
    p0 = np.zeros(len(states)); p0[index[(x0,)]] = 1.0
    pT = linalg.expm(Q * dt * n) @ p0
    exp = np.zeros(top + 1)
    for s, pr in zip(states, pT):
        exp[s[0]] += pr
    obs = np.bincount(x, minlength=top + 1)[:top + 1]
    pval, _, _ = refmath.chisquare_pvalue(obs, exp * x.size)
    assert pval > 0.01
    mean = float(np.sum(np.arange(top + 1) * exp))
    var = float(np.sum((np.arange(top + 1) - mean) ** 2 * exp))
    assert abs(x.mean() - mean) < 3 * math.sqrt(var / x.size)


@pytest.mark.parametrize("w,h,T", [(4, 4, 0.5), (3, 2, 0.3), (2, 1, 0.2)])
def test_diffusion_single_molecule_law(oracle_lib, w, h, T):
    D, n0, dt = 1.0, 12, 0.1
    steps = int(round(T / dt))
    side = 80
    p = W.pure_diffusion(w, h, D, 0, n0, nx=side, ny=side, dt=dt, n_steps=steps)
    x = oracle_lib.run(p, dt, steps).counts.reshape(side * side, w * h).astype(np.int64)
    assert np.all(x.sum(axis=1) == n0)  # diffusion conserves each cell's total
    # generator of one molecule: rate D to each mesh neighbour
    V = w * h
    Q = np.zeros((V, V))
    for v in range(V):
        vx, vy = v % w, v // w
        for dx, dy in [(-1, 0), (1, 0), (0, -1), (0, 1)]:
            if 0 <= vx + dx < w and 0 <= vy + dy < h:
                u = (vy + dy) * w + vx + dx
                Q[u, v] += D
                Q[v, v] -= D
    e0 = np.zeros(V); e0[0] = 1.0
    pv = linalg.expm(Q * T) @ e0
    N = x.shape[0]
    for v in range(V):
        mean, var = n0 * pv[v], n0 * pv[v] * (1 - pv[v])
        assert abs(x[:, v].mean() - mean) < 3.5 * math.sqrt(var / N) + 1e-12
        obs = np.bincount(x[:, v], minlength=n0 + 1)
        pval, _, _ = refmath.chisquare_pvalue(obs, stats.binom.pmf(np.arange(n0 + 1), n0, pv[v]) * N)
        assert pval > 0.001


# ---------------------------------------------------------------------------
# Split scheme vs brute-force CME
# ---------------------------------------------------------------------------


def test_split_scheme_matches_split_cme(oracle_lib):
    init = np.array([[3, 1, 0, 0, 0], [1, 3, 0, 0, 0]], np.int32)
    p = _two_cell_nd5(c4=0.7, c7=0.8, c8=0.5, c9=1.5, init=init)
    dt, n = 0.6, 3
    states, index, pv, _ = _split_law(p, dt, n)
    _, _, pv_rev, _ = _split_law(p, dt, n, order="s_then_chi")
    N = 20000
    obs = np.zeros(len(states))
    for sim in range(N):
        p["sim_id"] = sim
        r = oracle_lib.run(p, dt, n)
        obs[index[tuple(int(v) for v in r.counts)]] += 1
    pval, _, _ = refmath.chisquare_pvalue(obs, pv * N)
    assert pval > 0.01
    # the reversed operator order is a different law, and the sample sees it
    assert np.abs(pv - pv_rev).sum() > 0.05
    pval_rev, _, _ = refmath.chisquare_pvalue(obs, pv_rev * N)
    assert pval_rev < 1e-6


def test_split_scheme_converges_to_unsplit_cme():
    """Lie splitting error at fixed T shrinks ~ linearly in dt (the paper's
    premise that the split solution converges as dt -> 0)."""
    init = np.array([[3, 1, 0, 0, 0], [1, 3, 0, 0, 0]], np.int32)
    p = _two_cell_nd5(c4=0.7, c7=0.8, c8=0.5, c9=1.5, init=init)
    T = 1.2
    errs = []
    for n in (2, 4, 8, 16):
        states, index, pv, Q = _split_law(p, T / n, n)
        x0 = np.zeros(len(states)); x0[index[tuple(int(v) for v in init.ravel())]] = 1.0
        exact = linalg.expm(Q * T) @ x0
        errs.append(np.abs(pv - exact).sum())
    for a, b in zip(errs, errs[1:]):
        assert b < a
        assert 1.6 < a / b < 2.4  # first order


def test_split_scheme_with_voxels_and_faces(oracle_lib):
    """Two 2x1-voxel cells side by side (square lattice): S couples only the
    facing voxels (right voxel of the left cell, left voxel of the right
    cell); molecules diffuse between the two voxels of a cell."""
    m = W.model_tr()
    Dd = 0.9
    init = np.array([[1, 1, 0], [2, 0, 0],    # cell 0: voxel 0, voxel 1
                     [0, 2, 0], [1, 1, 0]], np.int32)  # cell 1
    p = W.make_problem(m, lattice=0, nx=2, ny=1, mesh_w=2, mesh_h=1, rates=[],
                       trans_rate=1.3, diffusion=Dd, init_counts=init, seed=41)
    S = 3
    dt, n = 0.5, 2

    def chi(s):
        out = []
        for cell in range(2):
            for v in range(2):
                for q in range(S):
                    c = s[(cell * 2 + v) * S + q]
                    if c:
                        ns = list(s)
                        ns[(cell * 2 + v) * S + q] -= 1
                        ns[(cell * 2 + (1 - v)) * S + q] += 1
                        out.append((Dd * c, tuple(ns)))
        return out

    def sig(s):
        out = []
        A, B = (0, 1), (1, 0)  # (cell, voxel) facing each other
        for recv, send in ((A, B), (B, A)):
            ri, si = (recv[0] * 2 + recv[1]) * S, (send[0] * 2 + send[1]) * S
            h = s[ri + 0] * s[si + 1]
            if h:
                ns = list(s)
                ns[ri + 0] -= 1; ns[si + 1] -= 1; ns[ri + 2] += 1
                out.append((1.3 * h, tuple(ns)))
        return out

    x0 = tuple(int(v) for v in init.ravel())
    states, index = refmath.enumerate_states(x0, lambda s: chi(s) + sig(s))
    Ec = linalg.expm(refmath.generator(states, index, chi) * dt)
    Es = linalg.expm(refmath.generator(states, index, sig) * dt)
    pv = np.zeros(len(states)); pv[index[x0]] = 1.0
    for _ in range(n):
        pv = Es @ (Ec @ pv)
    N = 15000
    obs = np.zeros(len(states))
    for sim in range(N):
        p["sim_id"] = sim
        r = oracle_lib.run(p, dt, n)
        obs[index[tuple(int(v) for v in r.counts)]] += 1
    pval, _, _ = refmath.chisquare_pvalue(obs, pv * N)
    assert pval > 0.01


# ---------------------------------------------------------------------------
# Invariants and step bookkeeping
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("lattice,mesh", [(1, (4, 4)), (0, (3, 2)), (1, (1, 1)), (1, (2, 2))])
def test_notch_conservation(oracle_lib, lattice, mesh):
    """With production and degradation off (r0-r3, r5, r6), N+C+I+R is
    conserved per cell and D+C+I+R per tissue."""
    p = W.random_problem(5, lattice=lattice, nx=5, ny=4, model="nd5", mesh=mesh,
                         rate_lo=-1.0, rate_hi=1.0, dt=0.1, n_steps=6)
    p["rates"][[0, 1, 2, 3, 5, 6]] = 0.0
    r = oracle_lib.run(p, p["dt"], p["n_steps"])
    assert r.s_events > 0 and r.chi_events > 0
    S = 5
    V = mesh[0] * mesh[1]
    x0 = p["init_counts"].reshape(-1, V, S).astype(np.int64)
    x1 = r.counts.reshape(-1, V, S).astype(np.int64)
    assert x1.min() >= 0
    N, D, I, R, Cc = range(5)
    per_cell = lambda x: x[:, :, [N, Cc, I, R]].sum(axis=(1, 2))
    assert np.array_equal(per_cell(x0), per_cell(x1))
    tissue = lambda x: x[:, :, [D, Cc, I, R]].sum()
    assert tissue(x0) == tissue(x1)


def test_chunking_and_resume_identity(oracle_lib):
    p = W.random_problem(7, lattice=1, nx=4, ny=3, model="nd5", mesh=(4, 4), dt=0.05, n_steps=6)
    full = oracle_lib.run(p, p["dt"], 6, trace=True)
    a = oracle_lib.run(p, p["dt"], 2, trace=True)
    b = oracle_lib.run(p, p["dt"], 4, counts=a.counts, start_step=2, trace=True)
    assert np.array_equal(full.counts, b.counts)
    assert full.chi_events == a.chi_events + b.chi_events
    assert np.array_equal(full.chi_trace_t[2:], b.chi_trace_t)
    assert np.array_equal(full.s_trace_events[:2], a.s_trace_events)


def test_thread_count_does_not_change_bits(oracle_lib):
    p = W.random_problem(8, lattice=1, nx=6, ny=5, model="nd5", uneven=True, dt=0.05, n_steps=3)
    r1 = oracle_lib.run(p, p["dt"], 3, threads=1, trace=True)
    r4 = oracle_lib.run(p, p["dt"], 3, threads=4, trace=True)
    assert np.array_equal(r1.counts, r4.counts)
    assert np.array_equal(r1.chi_trace_t, r4.chi_trace_t)
    assert np.array_equal(r1.s_trace_t, r4.s_trace_t)


def test_event_cap_stops_a_unit(oracle_lib):
    p = W.birth_death(1e6, 0.0, 0, dt=1.0, n_steps=1)
    p["event_cap"] = 1000
    r = oracle_lib.run(p, 1.0, 1)
    assert r.capped and r.chi_events == 1000 and r.counts[0] == 1000


@pytest.mark.parametrize("margin,expect", [(0, True), (1, False), (-3, True), (1000, False)])
def test_range_flag_at_2_26(oracle_lib, margin, expect):
    """The range contract: a count reaching 2^26 flags the tissue while the
    simulation goes on.  Pinned by the textbook direct method on the same
    streams (int64 counts, no range check).  Under pure birth the
    propensity does not depend on the count, so each cell's births N_c over
    the unit interval are fixed by its draws alone: a first textbook run
    from zero gives them, and cells started at 2^26 - N_c - margin end
    exactly `margin` below 2^26 (margin 0: exactly at the limit, flagged;
    margin 1: one below, not flagged).  The oracle's counts are the
    textbook's and its flag is set exactly when a count reached 2^26."""
    p = W.birth_death(50.0, 0.0, 0, nx=3, ny=2, dt=1.0, n_steps=1, seed=29)
    births = refmath.textbook_v1(p, 1).astype(np.int64)
    assert births.min() > 20
    x0 = np.where(np.arange(6) == 4, (1 << 26) - births - margin, 1000 - births)
    q = dict(p, init_counts=x0.astype(np.int32).reshape(6, 1))
    want = refmath.textbook_v1(q, 1).astype(np.int64)
    assert want[4] == (1 << 26) - margin
    r = oracle_lib.run(q, 1.0, 1)
    assert np.array_equal(r.counts.astype(np.int64), want)
    assert r.chi_events == int(births.sum())
    assert r.overflow == bool((want >= (1 << 26)).any()) == expect
