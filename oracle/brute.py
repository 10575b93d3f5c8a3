"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Brute-force enumeration over every state of small instances (<= ~20 spins),
used to pin the oracle against exact mathematics:

* OPT of the constrained problem (Eq. primal_problem),
* LB_P = min_x E for the penalty energy (Eq. penalty_energy, Eq. min_E) and the
  critical penalty P_C above which LB_P = OPT (Sec. II-A),
* the dual function LB_L(lambda) = min_x L (Eq. min_L, Eq. dual_problem),
* the exact law of the quantised sequential Gibbs sampler after a run, and the
  Boltzmann law exp(-beta L) it should approach (Eq. Boltzmann_distrib).

Energies here are evaluated in the minimisation form of the paper,
f(x) = -profit(x)/s_f, with g(x) = (A_ext x - b)/s_g, as exact Fractions.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import oracle as O


def all_states(nbits: int) -> np.ndarray:
    idx = np.arange(1 << nbits, dtype=np.int64)
    return ((idx[:, None] >> np.arange(nbits)) & 1).astype(np.int64)


def opt_max(prog: O.Program):
    """Largest profit over feasible original assignments, and one argmax."""
    xs = all_states(prog.n)
    profit, feas = O.score(prog, np.concatenate(
        [xs, np.zeros((len(xs), prog.n_ext - prog.n), dtype=np.int64)], axis=1))
    if not feas.any():
        return None, None
    best = int(np.argmax(np.where(feas, profit, np.iinfo(np.int64).min)))
    return int(profit[best]), xs[best]


def ext_table(prog: O.Program):
    """(states, profit, g) for every extended state."""
    xs = all_states(prog.n_ext)
    profit = O.profit_ext(prog, xs)
    g = O.residual(prog, xs)
    return xs, profit, g


def lb_penalty(prog: O.Program, P: Fraction, table=None) -> Fraction:
    """min over extended states of -profit/s_f + P |g|^2 / s_g^2."""
    xs, profit, g = table if table is not None else ext_table(prog)
    P = Fraction(P)
    sq = (g * g).sum(axis=1)
    # scale by s_f s_g^2 P.denominator to compare integers
    val = (-profit * prog.s_g ** 2 * P.denominator + P.numerator * prog.s_f * sq)
    i = int(np.argmin(val))
    return Fraction(int(val[i]), prog.s_f * prog.s_g ** 2 * P.denominator)


def lagrangian_values(prog: O.Program, P: Fraction, lam, table=None):
    """Exact L_n for every extended state as Fractions (small instances only)."""
    xs, profit, g = table if table is not None else ext_table(prog)
    P = Fraction(P)
    lam = [Fraction(v) for v in lam]
    out = []
    for r in range(len(xs)):
        gr = [int(v) for v in g[r]]
        L = (Fraction(-int(profit[r]), prog.s_f) + P * Fraction(sum(v * v for v in gr), prog.s_g ** 2)
             + sum(l * Fraction(v, prog.s_g) for l, v in zip(lam, gr)))
        out.append(L)
    return out


def lb_lagrange(prog: O.Program, P: Fraction, lam, table=None):
    """(LB_L(lambda), g of one minimiser)."""
    tab = table if table is not None else ext_table(prog)
    vals = lagrangian_values(prog, P, lam, tab)
    i = min(range(len(vals)), key=lambda r: vals[r])
    return vals[i], [int(v) for v in tab[2][i]]


def p_critical(prog: O.Program, table=None) -> Fraction:
    """Smallest normalised P with LB_P = OPT:
    max over states with g != 0 of (OPT_min - f(x)) s_g^2 / (s_f |g|^2), at least 0."""
    opt, _ = opt_max(prog)
    xs, profit, g = table if table is not None else ext_table(prog)
    sq = (g * g).sum(axis=1)
    pc = Fraction(0)
    for r in np.nonzero(sq > 0)[0]:
        # f = -profit/s_f, OPT_min = -opt/s_f
        gain = int(profit[r]) - opt          # (OPT_min - f) * s_f
        if gain > 0:
            pc = max(pc, Fraction(gain * prog.s_g ** 2, prog.s_f * int(sq[r])))
    return pc


# ---------------------------------------------------------------------------
# exact law of the quantised sampler

def site_probabilities(prog: O.Program, lq):
    """p[t][i][s] = probability that sweep t sets spin i to 1 from state s,
    from the energy definition (not the sampler's field formula)."""
    xs = all_states(prog.n_ext)
    E = np.array([O.energy(prog, x, lq) for x in xs], dtype=object)
    theta = O.theta_table()
    nstates = len(xs)
    Z = np.zeros((prog.n_ext, nstates), dtype=object)
    for i in range(prog.n_ext):
        bit = 1 << i
        for s in range(nstates):
            Z[i, s] = -(E[s | bit] - E[s & ~bit])
    probs = []
    cache = {}
    for t in range(prog.T):
        key = prog.B[t]
        if key not in cache:
            pt = np.zeros((prog.n_ext, nstates))
            for i in range(prog.n_ext):
                for s in range(nstates):
                    pt[i, s] = theta[O.index_of(prog, Z[i, s], t) + O.THETA_HALF] / float(O.ONE24)
            cache[key] = pt
        probs.append(cache[key])
    return probs


def apply_site(dist: np.ndarray, i: int, p1: np.ndarray) -> np.ndarray:
    nstates = len(dist)
    bit = 1 << i
    s = np.arange(nstates)
    out = np.zeros_like(dist)
    np.add.at(out, s | bit, dist * p1)
    np.add.at(out, s & ~bit, dist * (1.0 - p1))
    return out


def exact_run_law(prog: O.Program, lq) -> np.ndarray:
    """Distribution of the final state of one annealing run started at x = 0
    (state index = sum_i x_i 2^i)."""
    probs = site_probabilities(prog, lq)
    dist = np.zeros(1 << prog.n_ext)
    dist[0] = 1.0
    for t in range(prog.T):
        for i in range(prog.n_ext):
            dist = apply_site(dist, i, probs[t][i])
    return dist


def sweep_matrix(prog: O.Program, lq, t: int) -> np.ndarray:
    """Transition matrix of one full sweep at grid value B_t."""
    probs = site_probabilities(prog, lq)[t]
    nstates = 1 << prog.n_ext
    K = np.eye(nstates)
    for i in range(prog.n_ext):
        K = np.stack([apply_site(K[r], i, probs[i]) for r in range(nstates)])
    return K


def stationary(K: np.ndarray) -> np.ndarray:
    w, v = np.linalg.eig(K.T)
    j = int(np.argmin(np.abs(w - 1.0)))
    pi = np.real(v[:, j])
    pi = np.abs(pi)
    return pi / pi.sum()


def boltzmann(prog: O.Program, lq, beta: Fraction) -> np.ndarray:
    xs = all_states(prog.n_ext)
    E = np.array([float(Fraction(O.energy(prog, x, lq), prog.D)) for x in xs])
    w = np.exp(-float(beta) * (E - E.min()))
    return w / w.sum()
