"""Pins of the oracle parts every other check rests on, against definitions
written out here from the paper, independently of the oracle's own code:

* energy(): D * L_n, with L_n the normalised Lagrangian of Eq. penalty_energy
  and Eq. Lagrange_energy evaluated term by term from the raw problem data
  (profits, weights, capacities and the slack bits of Sec. IV-A), over every
  state of small QKP and MKP instances, at several P and lambda of both signs;
* lambda_step(): the multiplier step of Algorithm 1 recomputed with exact
  rationals, with half-way ties of both signs whose expected values are
  written as literals (round half away from zero, the reading the oracle
  states), and the saturation bound;
* best_update(): the best feasible record (Algorithm 1 keeps the feasible
  samples and returns the best), on hand-built rounds that separate
  "earliest round, then lowest replica" from every other tie order.
"""
from fractions import Fraction
from itertools import product
from math import floor

import numpy as np
import pytest

from oracle import brute as BF
from oracle import oracle as O
from paper_2501_04971_amd import generators as G


# ---------------------------------------------------------------- energy

def _lagrangian_by_definition(prob, P, lam, x_ext):
    """L_n(x) = -profit(x)/s_f + P |g|^2/s_g^2 + sum_k lam_k g_k/s_g from the raw
    data, with g_k = sum_i a_ki x_i + slack_k - b_k and slack_k the value of the
    bitlen(b_k) slack bits of constraint k (after the originals, constraint by
    constraint, least significant first)."""
    n, m = prob.n, prob.m
    a = [[int(v) for v in row] for row in np.asarray(prob.weight).reshape(m, n)]
    b = [int(v) for v in np.asarray(prob.capacity).reshape(m)]
    x = [int(v) for v in x_ext]
    if prob.kind == G.KIND_QKP:
        p = [[int(v) for v in row] for row in np.asarray(prob.profit).reshape(n, n)]
        entries = [abs(v) for row in p for v in row]
        profit = sum(p[i][i] * x[i] for i in range(n))
        profit += sum(p[i][j] * x[i] * x[j] for i in range(n) for j in range(i + 1, n))
    else:
        c = [int(v) for v in np.asarray(prob.profit).reshape(n)]
        entries = [abs(v) for v in c]
        profit = sum(c[i] * x[i] for i in range(n))
    s_f = max([1] + entries)
    s_g = max([1] + [v for row in a for v in row] + b)
    pos = n
    g = []
    for k in range(m):
        q = b[k].bit_length()
        slack = sum(x[pos + j] << j for j in range(q))
        pos += q
        g.append(sum(a[k][i] * x[i] for i in range(n)) + slack - b[k])
    assert pos == len(x)
    L = Fraction(-profit, s_f) + Fraction(P) * Fraction(sum(v * v for v in g), s_g * s_g)
    L += sum(Fraction(l) * Fraction(v, s_g) for l, v in zip(lam, g))
    return L, 256 * s_f * s_g * s_g


def _pin_instances():
    out = []
    for seed in range(3):
        out.append(G.tiny(5, 1, True, G.rng_for(980, seed), pmax=9, wmax=6))
    for seed in range(3):
        out.append(G.tiny(4, 1 + seed, False, G.rng_for(981, seed), pmax=9, wmax=5))
    # negative pair profits too (the encoding allows them)
    q = G.tiny(5, 1, True, G.rng_for(982, 0), pmax=7, wmax=6)
    q.profit = (q.profit.astype(np.int64) - 3).astype(np.int32)
    out.append(q)
    return out


@pytest.mark.parametrize("which", range(7))
def test_energy_is_the_normalised_lagrangian(which):
    """energy(x, lq) = D * L_n(x) for every extended state, P = pq/256 and
    lambda = lq/256 of both signs; a slip in any one term (the lambda term over
    s_g^2, the penalty over s_g, a slack bit weighted wrongly) breaks it."""
    prob = _pin_instances()[which]
    rng = np.random.default_rng(100 + which)
    for pq in [0, 37, 3 * 256, 1000]:
        prog = O.build_program(prob, G.Params(replicas=1, sweeps=2, p_q=pq))
        assert prog.n_ext <= 13
        for trial in range(2):
            lq = [int(v) for v in rng.integers(-900, 900, size=prog.m)]
            if trial == 1:
                lq = [-v if k % 2 else v for k, v in enumerate(lq)]
            states = BF.all_states(prog.n_ext)
            pick = states if len(states) <= 1024 else states[rng.choice(len(states), 1024, replace=False)]
            for x in pick:
                L, D = _lagrangian_by_definition(prob, Fraction(pq, 256), [Fraction(v, 256) for v in lq], x)
                assert prog.D == D
                assert O.energy(prog, x, lq) == D * L


def test_energy_agrees_with_the_enumeration_checker():
    """The same identity against brute.lagrangian_values, which the duality pins use."""
    for prob in _pin_instances()[:4]:
        prog = O.build_program(prob, G.Params(replicas=1, sweeps=2, p_q=300))
        lq = [-517 + 40 * k for k in range(prog.m)]
        vals = BF.lagrangian_values(prog, Fraction(300, 256), [Fraction(v, 256) for v in lq])
        for x, L in zip(BF.all_states(prog.n_ext), vals):
            assert O.energy(prog, x, lq) == prog.D * L


# ---------------------------------------------------------------- lambda step

def _tie_prog():
    prog = O.build_program(G.family0(0), G.Params(replicas=1))
    # eta = s_g / 2^33 makes the accumulator step 2^32 eta G / (R s_g) = G / 2
    prog.eta = Fraction(prog.s_g, 1 << 33)
    return prog


@pytest.mark.parametrize("G_,delta", [(5, 3), (-5, -3), (3, 2), (-3, -2), (1, 1), (-1, -1),
                                      (4, 2), (-4, -2), (0, 0)])
def test_lambda_step_half_way_ties_go_away_from_zero(G_, delta):
    """Accumulator step round(G/2) at exact halves: half away from zero (half to
    even would give 2 for 5/2 and 0 for 1/2; half up would give -2 for -5/2)."""
    prog = _tie_prog()
    acc, _ = O.lambda_step(prog, [1 << 40], [G_], 1)
    assert acc == [(1 << 40) + delta]


@pytest.mark.parametrize("acc,lq", [(1 << 23, 1), (-(1 << 23), -1), (3 << 23, 2), (-(3 << 23), -2),
                                    (5 << 23, 3), (-(5 << 23), -3), ((1 << 23) - 1, 0),
                                    (-(1 << 23) + 1, 0), ((1 << 24) + (1 << 23) - 1, 1)])
def test_multiplier_grid_rounding_ties(acc, lq):
    """lambda_q = round(acc / 2^24) half away from zero, from the accumulator alone."""
    prog = _tie_prog()
    new_acc, got = O.lambda_step(prog, [acc], [0], 1)
    assert new_acc == [acc] and got == [lq]


def test_lambda_step_exact_rationals():
    """Random steps recomputed with Fractions: acc += round(2^32 eta G/(R s_g)),
    lambda_q = round(acc/2^24), both half away from zero, clamped at lq_max 2^24."""
    rng = np.random.default_rng(31)

    def rha(v: Fraction) -> int:
        a = abs(v)
        q = floor(a)
        q += 1 if a - q >= Fraction(1, 2) else 0
        return q if v >= 0 else -q

    for fam, R in [(0, 64), (1, 1024), (1, 3)]:
        prob = G.family0(0) if fam == 0 else G.family1(0)
        prog = O.build_program(prob, G.Params(replicas=R, eta=Fraction(int(rng.integers(1, 50)),
                                                                         int(rng.integers(1, 400)))))
        cap = prog.lq_max << 24
        acc = [int(v) for v in rng.integers(-(1 << 40), 1 << 40, size=prog.m)]
        for _ in range(60):
            G_ = [int(v) for v in rng.integers(-R * 3000, R * 3000, size=prog.m)]
            new_acc, lq = O.lambda_step(prog, acc, G_, R)
            for a0, gk, a1, l1 in zip(acc, G_, new_acc, lq):
                step = rha(Fraction(1 << 32) * prog.eta * gk / (R * prog.s_g))
                assert a1 == max(-cap, min(cap, a0 + step))
                assert l1 == rha(Fraction(a1, 1 << 24))
            acc = new_acc


def test_diminishing_step_literal_values():
    """eta_k = eta H / (H + k): with eta = s_g / 2^32 and H = 4 the accumulator
    step for G = 30 after rounds k = 0..5 is 30 * 4/(4 + k) rounded half away
    from zero: 30, 24, 20, 17.142.. -> 17, 15, 13.33.. -> 13 (literals)."""
    prog = O.build_program(G.family0(0), G.Params(replicas=1, eta_decay=4))
    prog.eta = Fraction(prog.s_g, 1 << 32)
    assert prog.eta_decay == 4
    acc = [0]
    steps = []
    for k in range(6):
        new, _ = O.lambda_step(prog, acc, [30], 1, k=k)
        steps.append(new[0] - acc[0])
        acc = new
    assert steps == [30, 24, 20, 17, 15, 13]
    # negative residual sums mirror them; a constant step ignores k
    new, _ = O.lambda_step(prog, [0], [-30], 1, k=3)
    assert new == [-17]
    prog.eta_decay = 0
    assert O.lambda_step(prog, [0], [30], 1, k=5)[0] == [30]


def test_diminishing_step_sum_diverges_and_squares_converge():
    """The step sizes meet the conditions of the surrogate subgradient method:
    sum_k eta_k grows like H log K without bound, sum eta_k^2 stays below
    eta^2 H (H + 1)."""
    prog = O.build_program(G.family0(0), G.Params(replicas=1, eta=Fraction(1, 2), eta_decay=8))
    s1 = s2 = Fraction(0)
    for k in range(4000):
        e = O.step_size(prog, k)
        assert e == Fraction(1, 2) * Fraction(8, 8 + k)
        s1 += e
        s2 += e * e
    assert s1 > Fraction(1, 2) * 8 * 6  # H (ln(4008/8) ~ 6.2) eta
    assert s2 < Fraction(1, 4) * 8 * 9


def test_diminishing_step_index_is_capped():
    prog = O.build_program(G.family0(0), G.Params(replicas=64, eta_decay=16))
    lam_den = prog.eta.denominator * 64 * prog.s_g
    assert prog.eta_kcap == min(((1 << 62) - 1) // lam_den - 16, (1 << 31) - 1)
    assert O.step_size(prog, prog.eta_kcap + 1000) == O.step_size(prog, prog.eta_kcap)
    assert O.step_size(prog, -3) == prog.eta  # before any round: k = 0


def test_saturation_mask_is_sticky():
    prog = O.build_program(G.family0(0), G.Params(replicas=1))
    cap = prog.lq_max << 24
    assert O.saturation_mask([cap - 1], cap, 0) == 0
    assert O.saturation_mask([-cap], cap, 0) == 1
    assert O.saturation_mask([0, cap], cap, 1) == 3


# ---------------------------------------------------------------- best record

def test_best_record_takes_the_earliest_round_then_the_lowest_replica():
    """Round 0: replica 1 infeasible at 9, replica 2 feasible at 9.  Round 1:
    replicas 0 and 1 feasible at 9 and an infeasible 12.  The best is (9, round 0,
    replica 2): 'lowest replica first' would give round 1 replica 0, 'latest'
    round 1 replica 1, and ignoring feasibility 12."""
    x = np.arange(12).reshape(3, 4) % 2
    best = O.best_update(None, 0, np.array([5, 9, 9]), np.array([True, False, True]), x)
    assert best[:3] == (9, 0, 2)
    best = O.best_update(best, 1, np.array([9, 9, 12]), np.array([True, True, False]), x + 1)
    assert best[:3] == (9, 0, 2) and (best[3] == x[2]).all()
    # a strictly larger profit in a later round replaces it; its lowest replica wins
    best = O.best_update(best, 2, np.array([7, 10, 10]), np.array([True, True, True]), x)
    assert best[:3] == (10, 2, 1)
    # nothing feasible keeps the record
    assert O.best_update(best, 3, np.array([99, 99, 99]), np.zeros(3, bool), x)[:3] == (10, 2, 1)
    assert O.best_update(None, 0, np.array([1, 2]), np.zeros(2, bool), x[:2]) is None


def test_saim_best_matches_its_round_logs():
    """saim()'s best equals the first (round, replica) in order among the feasible
    samples of largest profit in its own per-round logs."""
    prob = G.tiny(6, 1, True, G.rng_for(983, 0), pmax=9, wmax=7)
    par = G.Params(replicas=40, sweeps=30, beta=Fraction(4), eta=Fraction(3), p_q=256)
    res = O.saim(prob, par, 4, nthreads=2)
    cands = [(int(e["profit"][r]), -k, -r) for k, e in enumerate(res["rounds"])
             for r in range(par.replicas) if e["feasible_mask"][r]]
    top = max(cands)
    assert res["best"][:3] == (top[0], -top[1], -top[2])
    ties = [c for c in cands if c[0] == top[0]]
    assert len(ties) > 1  # the tie rule decided it


# ---------------------------------------------------------------- counter bound

def test_philox_counter_word_does_not_wrap():
    """T * ceil(N_ext/4) must fit the 32-bit counter word (t ceil(N_ext/4) + i/4):
    otherwise later sweeps would replay earlier draws."""
    prob = G.family0(0)
    prog = O.build_program(prob, G.Params(replicas=1, sweeps=10))
    nq = (prog.n_ext + 3) // 4
    T_ok = (1 << 32) // nq
    assert T_ok * nq <= 1 << 32 < (T_ok + 1) * nq
    with pytest.raises(O.OracleRangeError):
        O.build_program(prob, G.Params(replicas=1, sweeps=T_ok + 1))
