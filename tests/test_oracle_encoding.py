"""Pins of the oracle's encoding against the paper's definitions and exact
mathematics (brute-force enumeration over small instances)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute as BF
from oracle import oracle as O
from paper_2501_04971_amd import generators as G

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def tiny_programs():
    out = []
    for seed in range(6):
        rng = G.rng_for(900, seed)
        quad = seed % 2 == 0
        m = 1 if quad else 1 + seed % 3
        n = 6 if quad else 5
        prob = G.tiny(n, m, quad, rng, pmax=9, wmax=7)
        prog = O.build_program(prob, G.Params(replicas=1, sweeps=4, beta=Fraction(3)))
        if prog.n_ext <= 14:
            out.append(prog)
    assert len(out) >= 4
    return out


def test_slack_encoding_equivalence():
    """x is feasible iff some slack assignment makes every residual zero (Sec. IV-A)."""
    for prog in tiny_programs():
        xs = BF.all_states(prog.n_ext)
        g = O.residual(prog, xs)
        zero = (g == 0).all(axis=1)
        orig = xs[:, :prog.n]
        code = (orig << np.arange(prog.n)).sum(axis=1)
        reach = set(int(c) for c in code[zero])
        for c in range(1 << prog.n):
            x = ((c >> np.arange(prog.n)) & 1).astype(np.int64)
            feasible = bool(((prog.A[:, :prog.n] @ x) <= prog.b).all())
            assert feasible == (c in reach)
        # Q_k = floor(log2 b_k + 1): the slack range covers [0, b_k] and no more bits
        for k, q in enumerate(prog.Q):
            assert (1 << q) - 1 >= prog.b[k]
            assert q == 0 or (1 << (q - 1)) <= prog.b[k]


def test_penalty_lower_bound_and_critical_value():
    """LB_P <= OPT for any P, and LB_P = OPT exactly when P >= P_C (Sec. II-A)."""
    for prog in tiny_programs():
        opt, _ = BF.opt_max(prog)
        opt_min = Fraction(-opt, prog.s_f)
        tab = BF.ext_table(prog)
        pc = BF.p_critical(prog, tab)
        for P in [Fraction(0), pc / 10, pc / 2, pc, pc * 2 + 1]:
            assert BF.lb_penalty(prog, P, tab) <= opt_min
        assert BF.lb_penalty(prog, pc, tab) == opt_min
        assert BF.lb_penalty(prog, pc * 2 + 1, tab) == opt_min
        if pc > 0:
            # a sub-critical penalty (e.g. 0.1 P_C) leaves a gap: the minimiser is infeasible
            assert BF.lb_penalty(prog, pc / 10, tab) < opt_min
            assert BF.lb_penalty(prog, pc * Fraction(999, 1000), tab) < opt_min


def test_weak_duality_concavity_supergradient():
    """LB_L(lambda) <= OPT; LB_L is concave in lambda; g at a minimiser is a
    supergradient (Sec. II-B, Sec. III-A)."""
    rng = np.random.default_rng(5)
    for prog in tiny_programs()[:4]:
        opt, _ = BF.opt_max(prog)
        opt_min = Fraction(-opt, prog.s_f)
        tab = BF.ext_table(prog)
        P = BF.p_critical(prog, tab) / 10
        lams = [[Fraction(int(v), 4) for v in rng.integers(-40, 40, size=prog.m)] for _ in range(5)]
        vals = {}
        for lam in lams:
            lb, gbar = BF.lb_lagrange(prog, P, lam, tab)
            vals[tuple(lam)] = (lb, gbar)
            assert lb <= opt_min
        for a in lams:
            for b in lams:
                mid = [(u + v) / 2 for u, v in zip(a, b)]
                lm, _ = BF.lb_lagrange(prog, P, mid, tab)
                assert lm >= (vals[tuple(a)][0] + vals[tuple(b)][0]) / 2
                lb_a, g_a = vals[tuple(a)]
                # supergradient inequality in normalised units g/s_g
                bound = lb_a + sum(Fraction(gk, prog.s_g) * (v - u) for gk, u, v in zip(g_a, a, b))
                assert vals[tuple(b)][0] <= bound


def test_lagrange_term_closes_the_gap():
    """At a sub-critical P there is a lambda whose Lagrangian minimum is the
    constrained optimum's value for some instance (Fig. 2 idea): the dual
    bound max_lambda LB_L exceeds LB_P."""
    improved = 0
    for prog in tiny_programs():
        tab = BF.ext_table(prog)
        pc = BF.p_critical(prog, tab)
        if pc == 0:
            continue
        P = pc / 10
        lbp = BF.lb_penalty(prog, P, tab)
        best = max(BF.lb_lagrange(prog, P, [Fraction(v, 2)] * prog.m, tab)[0] for v in range(0, 60, 3))
        assert best >= lbp
        improved += best > lbp
    assert improved >= 1


def test_penalty_rule_counts_slack_spins():
    """P = 2dN with d = 0.5, N = 300 + 13 slack spins gives 313 (Sec. IV-A)."""
    gold = GOLD["penalty_rule_qkp"]
    for idx in range(50):
        prob = G.qkp(gold["n"], Fraction(gold["density"]), G.rng_for(77, idx))
        if int(prob.capacity[0]).bit_length() == gold["slack_bits"]:
            break
    else:
        pytest.fail("no instance with the required capacity bit length")
    prog = O.build_program(prob, G.Params(alpha=Fraction(gold["alpha"])))
    assert prog.n_ext == gold["n"] + gold["slack_bits"]
    assert Fraction(prog.pq, 256) == gold["P"]


def test_penalty_rule_mkp_density():
    """MKP: d = 2/(N+1) and P = 5dN is about 10 (Sec. IV-B, Fig. 5)."""
    gold = GOLD["penalty_rule_mkp"]
    prob = G.mkp(gold["n"], gold["m"], G.rng_for(78, 0))
    prog = O.build_program(prob, G.Params(alpha=Fraction(gold["alpha"])))
    assert abs(prog.pq / 256 - gold["P"]) < gold["tolerance"]


def test_table1_defaults_used_by_workloads():
    """Where a workload leaves a setting open, Table 1's value for that kind is used."""
    t1 = GOLD["table1"]
    _, par1, _ = G.workload(1)
    assert par1.alpha == t1["MKP"]["alpha"] and par1.beta == t1["MKP"]["beta_max"]
    assert par1.eta == Fraction(t1["MKP"]["eta"])
    _, par0, _ = G.workload(0)
    assert par0.alpha == t1["QKP"]["alpha"]


def test_mcs_accounting():
    """Sample budgets of Sec. IV-A: 2e6 MCS for SAIM; 100x and 7,500x ratios."""
    gold = GOLD["mcs_accounting"]
    saim = gold["saim"][0] * gold["saim"][1]
    assert saim == 2_000_000
    assert gold["best_sa"][0] * gold["best_sa"][1] // saim == gold["ratio_best_sa"]
    assert gold["pt_da"][0] * gold["pt_da"][1] // saim == gold["ratio_pt_da"]


def test_scales_and_bounds_on_workloads():
    """Normalisation maxima (Sec. IV-A) and the int64 budget on every workload family."""
    for cfg in (0, 1, 2):
        prob, par, _ = G.workload(cfg)
        prog = O.build_program(prob, par)
        if prob.kind == G.KIND_QKP:
            assert prog.s_f == int(np.abs(np.asarray(prob.profit)).max())
        else:
            assert prog.s_f == int(np.asarray(prob.profit).max())
        assert prog.s_g == max(int(np.asarray(prob.weight).max()), int(np.asarray(prob.capacity).max()))
        assert prog.D == 256 * prog.s_f * prog.s_g ** 2
        assert (1 << 30) <= prog.B[-1] < (1 << 31)
        assert prog.B[0] == 0 and prog.lq_max >= 256
    for idx in range(1, 24, 2):   # the MKP half of the mixed batch, including N=500, M=30
        prob, par, _ = G.workload(3, idx)
        prog = O.build_program(prob, par)
        assert prog.lq_max >= 256


def test_score_matches_pairwise_definition():
    """profit = sum_i h_i x_i + sum_{i<j} W_ij x_i x_j and A x <= b, by explicit loops."""
    rng = np.random.default_rng(3)
    prob = G.qkp(30, Fraction(1, 2), G.rng_for(79, 0))
    prog = O.build_program(prob, G.Params())
    x = rng.integers(0, 2, size=(20, prog.n_ext))
    profit, feas = O.score(prog, x)
    P = np.asarray(prob.profit, dtype=np.int64)
    for r in range(20):
        s = 0
        for i in range(prog.n):
            for j in range(i, prog.n):
                s += int(P[i, j]) * int(x[r, i]) * int(x[r, j])
        assert s == profit[r]
        w = sum(int(prob.weight[0, i]) * int(x[r, i]) for i in range(prog.n))
        assert feas[r] == (w <= int(prob.capacity[0]))
