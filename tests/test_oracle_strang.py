"""Pins for the oracle's Strang splitting (G. Strang 1968, symmetric
splitting): each step is chi over dt/2 (counter tag 0), S over dt, chi over
dt/2 (tag 2).  The paper's framework rests on the modules being run one
after the other with a solution that converges as dt -> 0 (section "A
parallel framework for multiscale simulation of cells", design assumptions)
and leaves the accuracy/performance trade-off of dt to future work
(Discussion); the symmetric scheme is the second-order member of that
family.  CPU only."""
import math

import numpy as np
from scipy import linalg, stats

import refmath
from paper_1806_10889_amd import workloads as W
from splitlaw import split_law, two_cell_nd5

INIT = np.array([[3, 1, 0, 0, 0], [1, 3, 0, 0, 0]], np.int32)


def _two_cell():
    return two_cell_nd5(c4=0.7, c7=0.8, c8=0.5, c9=1.5, init=INIT.copy())


def test_strang_matches_its_split_cme(oracle_lib):
    """The sampled law after n Strang steps is e^{Qc dt/2} e^{Qs dt}
    e^{Qc dt/2} applied n times; Lie's law is a different one, and the same
    sample rejects it."""
    p = _two_cell()
    p["scheme"] = "strang"
    dt, n = 0.6, 3
    states, index, pv, _ = split_law(p, dt, n, order="strang")
    _, _, pv_lie, _ = split_law(p, dt, n, order="chi_then_s")
    N = 20000
    obs = np.zeros(len(states))
    for sim in range(N):
        p["sim_id"] = sim
        r = oracle_lib.run(p, dt, n)
        obs[index[tuple(int(v) for v in r.counts)]] += 1
    pval, _, _ = refmath.chisquare_pvalue(obs, pv * N)
    assert pval > 0.01
    assert np.abs(pv - pv_lie).sum() > 0.05
    pval_lie, _, _ = refmath.chisquare_pvalue(obs, pv_lie * N)
    assert pval_lie < 1e-6


def test_strang_converges_second_order():
    """At fixed T the Strang law's distance to the unsplit CME shrinks ~ dt^2
    (Lie's ~ dt), and it is smaller than Lie's at every dt."""
    p = _two_cell()
    T = 1.2
    errs, lie = [], []
    for n in (4, 8, 16, 32):  # (n = 2 is still pre-asymptotic)
        states, index, pv, Q = split_law(p, T / n, n, order="strang")
        _, _, pl, _ = split_law(p, T / n, n, order="chi_then_s")
        x0 = np.zeros(len(states))
        x0[index[tuple(int(v) for v in INIT.ravel())]] = 1.0
        exact = linalg.expm(Q * T) @ x0
        errs.append(np.abs(pv - exact).sum())
        lie.append(np.abs(pl - exact).sum())
    for a, b in zip(errs, errs[1:]):
        assert 3.2 < a / b < 4.8  # second order
    assert all(s < l for s, l in zip(errs, lie))


def test_strang_halves_add_to_dt_birth_death_law(oracle_lib):
    """Without S the two halves are chi over dt/2 twice: by memorylessness
    the law at T = n dt is the birth-death transient law at T (a half over
    dt instead of dt/2 would put it at 2T)."""
    k, gamma, x0, dt, n = 5.0, 0.5, 20, 0.1, 10
    p = W.birth_death(k, gamma, x0, nx=100, ny=100, dt=dt, n_steps=n, seed=17)
    p["scheme"] = "strang"
    x = oracle_lib.run(p, dt, n).counts.astype(np.int64)
    t = dt * n
    q = math.exp(-gamma * t)
    mean = x0 * q + (k / gamma) * (1 - q)
    var = x0 * q * (1 - q) + (k / gamma) * (1 - q)
    assert abs(x.mean() - mean) < 3 * math.sqrt(var / x.size)
    pmf = np.convolve(stats.binom.pmf(np.arange(0, x0 + 1), x0, q),
                      stats.poisson.pmf(np.arange(0, 120), (k / gamma) * (1 - q)))[:120]
    pval, _, _ = refmath.chisquare_pvalue(np.bincount(x, minlength=120)[:120], pmf * x.size)
    assert pval > 0.01
    # and the law at 2T (a doubled half) is rejected
    q2 = math.exp(-gamma * 2 * t)
    mean2 = x0 * q2 + (k / gamma) * (1 - q2)
    assert abs(x.mean() - mean2) > 10 * math.sqrt(var / x.size)


def test_strang_trace_sums_halves_and_keeps_second_clock(oracle_lib):
    """The per-(cell, step) chi trace sums the events of both halves and
    keeps the second half's clock, which is below dt/2."""
    p = W.random_problem(41, lattice=1, nx=6, ny=5, model="nd5", mesh=(2, 2), dt=0.2,
                         n_steps=5)
    p["scheme"] = "strang"
    r = oracle_lib.run(p, p["dt"], 5, trace=True)
    assert r.chi_events > 1000 and r.s_events > 0
    assert int(r.chi_trace_events.sum()) == r.chi_events
    assert int(r.s_trace_events.sum()) == r.s_events
    t = r.chi_trace_t.view(np.float64)
    assert (t < p["dt"] * 0.5).all() and (t > 0).any()
    # a Lie run of the same problem is a different trajectory
    p2 = dict(p)
    p2["scheme"] = "lie"
    assert not np.array_equal(oracle_lib.run(p2, p["dt"], 5).counts, r.counts)
