"""The split process of a tiny closed two-cell tissue, solved exactly: the
chi and S generators of the 5-species network (reactions within each cell,
the trans reaction over the one edge) on the reachable state space, and the
law after n split steps by matrix exponentials (Lie in either order, or
Strang's symmetric splitting)."""
import numpy as np
from scipy import linalg

import refmath
from paper_1806_10889_amd import workloads as W


def two_cell_nd5(c4, c7, c8, c9, init):
    m = W.model_nd5()
    rates = np.zeros(9)
    rates[4], rates[7], rates[8] = c4, c7, c8
    return W.make_problem(m, lattice=0, nx=2, ny=1, mesh_w=1, mesh_h=1, rates=rates,
                          trans_rate=c9, diffusion=0.0, init_counts=init, seed=31)


def nd5_two_cell_generators(p):
    S = 5
    st = p["stoich"]
    rates = p["rates"]
    reac = p["reactants"]

    def chi(s):
        out = []
        for cell in range(2):
            x = s[cell * S:(cell + 1) * S]
            for r in range(p["n_reactions"]):
                a, b = reac[r]
                if rates[r] == 0:
                    continue
                if a < 0 and b < 0:
                    h = 1
                elif b < 0:
                    h = x[a]
                elif a == b:
                    h = x[a] * (x[a] - 1) // 2
                else:
                    h = x[a] * x[b]
                if h == 0:
                    continue
                ns = list(s)
                for q in range(S):
                    ns[cell * S + q] += int(st[r][q])
                out.append((rates[r] * h, tuple(ns)))
        return out

    tn, td, ti = p["trans_n"], p["trans_d"], p["trans_i"]

    def sig(s):
        out = []
        for recv, send in ((0, 1), (1, 0)):
            h = s[recv * S + tn] * s[send * S + td]
            if h:
                ns = list(s)
                ns[recv * S + tn] -= 1
                ns[send * S + td] -= 1
                ns[recv * S + ti] += 1
                out.append((p["trans_rate"] * h, tuple(ns)))
        return out

    def both(s):
        return chi(s) + sig(s)
    return chi, sig, both


def split_law(p, dt, n_steps, order="chi_then_s"):
    chi, sig, both = nd5_two_cell_generators(p)
    x0 = tuple(int(v) for v in p["init_counts"].ravel())
    states, index = refmath.enumerate_states(x0, both)
    Qc = refmath.generator(states, index, chi)
    Qs = refmath.generator(states, index, sig)
    Ec, Es = linalg.expm(Qc * dt), linalg.expm(Qs * dt)
    Eh = linalg.expm(Qc * (dt * 0.5))
    pv = np.zeros(len(states)); pv[index[x0]] = 1.0
    for _ in range(n_steps):
        if order == "chi_then_s":
            pv = Es @ (Ec @ pv)
        elif order == "s_then_chi":
            pv = Ec @ (Es @ pv)
        elif order == "strang":
            pv = Eh @ (Es @ (Eh @ pv))
        else:
            raise ValueError(order)
    return states, index, pv, Qc + Qs
