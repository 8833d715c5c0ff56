"""Independent reference mathematics for pinning the oracle (tests only).

Nothing here is shared with the oracle or the GPU library: a generic Philox
written for any word size, an exact fused multiply-add through rationals, a
textbook Gillespie direct method for well-mixed cells, and chemical-master-
equation generators solved with scipy's matrix exponential.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

# ---------------------------------------------------------------------------
# Generic Philox-4xW (Salmon et al., SC'11): any word size W, R rounds.
# ---------------------------------------------------------------------------


def philox4(ctr, key, W, M0, M1, W0, W1, rounds=10):
    mask = (1 << W) - 1
    x = [int(c) & mask for c in ctr]
    k = [int(key[0]) & mask, int(key[1]) & mask]
    for rnd in range(rounds):
        if rnd:
            k = [(k[0] + W0) & mask, (k[1] + W1) & mask]
        p0 = M0 * x[0]
        p1 = M1 * x[2]
        hi0, lo0 = p0 >> W, p0 & mask
        hi1, lo1 = p1 >> W, p1 & mask
        x = [hi1 ^ x[1] ^ k[0], lo1, hi0 ^ x[3] ^ k[1], lo0]
    return x


PHILOX4x64 = dict(W=64, M0=0xD2E7470EE14C6C93, M1=0xCA5A826395121157,
                  W0=0x9E3779B97F4A7C15, W1=0xBB67AE8584CAA73B)
PHILOX4x32 = dict(W=32, M0=0xD2511F53, M1=0xCD9E8D57, W0=0x9E3779B9, W1=0xBB67AE85)


def philox4x32(ctr, key):
    return philox4(ctr, key, **PHILOX4x32)


def uniforms(words):
    m1 = ((words[0] << 32) | words[1]) >> 11
    m2 = ((words[2] << 32) | words[3]) >> 11
    return (m1 + 1) / 2.0 ** 53, m2 / 2.0 ** 53


# ---------------------------------------------------------------------------
# Exact fused multiply-add: a*b + c rounded once (Fraction -> float rounds
# correctly to nearest).
# ---------------------------------------------------------------------------


def fma(a: float, b: float, c: float) -> float:
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def plog_py(x: float) -> float:
    """The project's log written again in Python, for the textbook SSA."""
    import math
    fr, e = math.frexp(x)
    m, k = fr * 2.0, e - 1
    if m > 1.4142135623730951:
        m, k = m * 0.5, k + 1
    f = m - 1.0
    s = f / (2.0 + f)
    z = s * s
    cs = [2.0 / (2 * l + 3) for l in range(12)]
    p = cs[11]
    for l in range(10, -1, -1):
        p = fma(p, z, cs[l])
    q = fma(s * z, p, 2.0 * s)
    ln2_hi = float.fromhex("0x1.62e42fefa39efp-1")
    ln2_lo = float.fromhex("0x1.abc9e3b39803fp-56")
    return fma(float(k), ln2_hi, fma(float(k), ln2_lo, q))


# ---------------------------------------------------------------------------
# Textbook direct method for tissues of well-mixed cells (V = 1), with the
# signalling operator on the square lattice; written from Gillespie's
# description, channels searched linearly.
# ---------------------------------------------------------------------------


def textbook_v1(problem, n_steps):
    p = problem
    nx, ny, S = p["nx"], p["ny"], p["n_species"]
    x = np.array(p["init_counts"], dtype=np.int64).reshape(nx * ny, S)
    R = p["n_reactions"]
    key = (p["seed"] & 0xFFFFFFFF, p["seed"] >> 32)
    dt = p["dt"]
    tn, td, ti = p["trans_n"], p["trans_d"], p["trans_i"]

    def props_cell(xc):
        out = []
        for r in range(R):
            a, b = p["reactants"][r]
            c = float(p["rates"][r])
            if a < 0 and b < 0:
                out.append(c)
            elif b < 0:
                out.append(c * float(int(xc[a])))
            elif a == b:
                out.append(c * float(int(xc[a]) * (int(xc[a]) - 1) // 2))
            else:
                out.append(c * float(int(xc[a]) * int(xc[b])))
        return out

    def pick(props, rr):
        acc = 0.0
        for k, a in enumerate(props):
            acc = acc + a
            if rr < acc and a > 0:
                return k
        return max(k for k, a in enumerate(props) if a > 0)

    def run_unit(unit, tag, step, props_fn, apply_fn):
        t, j = 0.0, 0
        while True:
            props = props_fn()
            a0 = 0.0
            for a in props:
                a0 = a0 + a
            if a0 == 0.0:
                return
            w = philox4x32((j, step, unit, (p["sim_id"] << 2) | tag), key)
            j += 1
            u1, u2 = uniforms(w)
            tau = (-plog_py(u1)) / a0
            if t + tau >= dt:
                return
            t = t + tau
            apply_fn(pick(props, u2 * a0))

    # edges of the square lattice: forward +x (colour x%2), +y (colour 2 + y%2)
    edges = []
    for col in range(4):
        d, par = divmod(col, 2)
        for i in range(nx * ny):
            cx, cy = i % nx, i // nx
            if (cx if d == 0 else cy) % 2 != par:
                continue
            if d == 0 and cx + 1 < nx:
                edges.append((col, i, i + 1))
            if d == 1 and cy + 1 < ny:
                edges.append((col, i, i + nx))
    for k in range(n_steps):
        step = p["start_step"] + k
        for c in range(nx * ny):
            def apply(r, c=c):
                x[c] += p["stoich"][r]
            run_unit(c, 0, step, lambda c=c: props_cell(x[c]), apply)
        if tn >= 0:
            for e, (col, i, j) in enumerate(edges):
                def props_e(i=i, j=j):
                    rate = float(p["trans_rate"])
                    return [rate * float(int(x[i, tn]) * int(x[j, td])),
                            rate * float(int(x[j, tn]) * int(x[i, td]))]

                def apply_e(ch, i=i, j=j):
                    a, b = (i, j) if ch == 0 else (j, i)
                    x[a, tn] -= 1
                    x[b, td] -= 1
                    x[a, ti] += 1
                run_unit(e, 1, step, props_e, apply_e)
    return x.astype(np.int32).ravel()


# ---------------------------------------------------------------------------
# Chemical master equation on an enumerated state space
# ---------------------------------------------------------------------------


def enumerate_states(x0, transitions, limit=200000):
    """BFS over states reachable from x0.  transitions(state) -> list of
    (rate, new_state).  Returns (states list, index dict)."""
    x0 = tuple(int(v) for v in x0)
    states = [x0]
    index = {x0: 0}
    q = 0
    while q < len(states):
        s = states[q]
        q += 1
        for rate, ns in transitions(s):
            if rate > 0 and ns not in index:
                index[ns] = len(states)
                states.append(ns)
                if len(states) > limit:
                    raise RuntimeError("state space too large")
    return states, index


def generator(states, index, transitions):
    """Dense CME generator Q (columns sum to zero): dp/dt = Q p."""
    n = len(states)
    Q = np.zeros((n, n))
    for a, s in enumerate(states):
        for rate, ns in transitions(s):
            if rate <= 0:
                continue
            b = index[ns]
            Q[b, a] += rate
            Q[a, a] -= rate
    return Q


def chisquare_pvalue(observed, expected, min_expected=5.0):
    """Pearson chi-square p-value after pooling bins with small expectation."""
    from scipy import stats
    observed = np.asarray(observed, float)
    expected = np.asarray(expected, float)
    order = np.argsort(expected)[::-1]
    obs_b, exp_b = [], []
    acc_o = acc_e = 0.0
    for k in order:
        acc_o += observed[k]
        acc_e += expected[k]
        if acc_e >= min_expected:
            obs_b.append(acc_o)
            exp_b.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 and exp_b:
        obs_b[-1] += acc_o
        exp_b[-1] += acc_e
    obs_b, exp_b = np.array(obs_b), np.array(exp_b)
    exp_b *= obs_b.sum() / exp_b.sum()
    stat = float(np.sum((obs_b - exp_b) ** 2 / exp_b))
    dof = max(len(obs_b) - 1, 1)
    return float(stats.chi2.sf(stat, dof)), stat, dof


def discrete_ks_pvalue(x, pmf, seed=12345):
    """KS p-value of integer sample x against pmf (support 0..len-1) via the
    randomised probability-integral transform u = F(x-1) + V pmf(x),
    V ~ U(0,1), which is exactly U(0,1) under the null."""
    from scipy import stats
    pmf = np.asarray(pmf, float)
    cdf_below = np.concatenate([[0.0], np.cumsum(pmf)])[:-1]
    x = np.asarray(x, int)
    assert x.min() >= 0 and x.max() < len(pmf)
    v = np.random.default_rng(seed).uniform(size=x.size)
    u = cdf_below[x] + v * pmf[x]
    return float(stats.kstest(u, "uniform").pvalue)
