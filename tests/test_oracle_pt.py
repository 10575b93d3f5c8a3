"""Parallel tempering as the Ising machine inside Algorithm 1 (the oracle's
version), pinned against mathematics it must satisfy:

* the exchange table is exp(j/256) on the 2^-8 grid (closed forms);
* the C core's energy, which the exchange compares, is the normalised
  Lagrangian of its definition (the Python energy, itself pinned to the
  Fraction form);
* the coldest replica's state after a run follows the exact law of the joint
  chain (two replicas, their sweep operators at the ladder temperatures and the
  Metropolis exchange), computed by enumeration; the same law with the
  exchange's sign reversed is rejected by the same samples;
* the multiplier step averages the chains' samples only."""
import os
from fractions import Fraction
from math import exp, floor

import numpy as np
import pytest

from oracle import brute as BF
from oracle import oracle as O
from paper_2501_04971_amd import generators as G

from test_oracle_sampler import _chi2_pvalue, _state_codes


def test_exchange_table_closed_form():
    X = O.exchange_table()
    assert len(X) == O.XLEN
    assert X[-1] == 1 << 24                      # exp(0)
    assert X[0] == 0                             # 2^24 exp(-18) = 0.25
    assert X[-1 - 256] == round((1 << 24) / np.e)  # exp(-1)
    assert all(a <= b for a, b in zip(X, X[1:]))
    for j in (-1, -100, -777, -3000):
        assert abs(X[j - 1] - (1 << 24) * exp(j / 256)) <= 0.5 + 1e-6


def _prog(prob, **kw):
    return O.build_program(prob, G.Params(**kw))


def test_c_energy_is_the_definition():
    prob = G.tiny(5, 1, True, G.rng_for(950, 0), pmax=7, wmax=6)
    prog = _prog(prob, replicas=8, sweeps=4, beta=Fraction(3), p_q=300, pt_slots=4)
    for lq in ([0], [517], [-900]):
        for x in BF.all_states(prog.n_ext):
            assert O.energy_c(prog, x, lq) == O.energy(prog, x, lq)


def _ladder_prog(prog, j):
    """A copy of prog whose single sweep runs at ladder value j."""
    import dataclasses
    return dataclasses.replace(prog, T=1, B=[prog.Bl[j]])


def _exact_pt2_law(prog, lq, sign=1):
    """Law of the state at the cold position after T sweeps of a two-replica
    chain started at x = 0 (exchange attempted after even sweeps only)."""
    n = 1 << prog.n_ext
    K = [BF.sweep_matrix(_ladder_prog(prog, j), lq, 0) for j in range(2)]
    E = [O.energy(prog, x, lq) for x in BF.all_states(prog.n_ext)]
    X = O.exchange_table()
    dB = prog.Bl[0] - prog.Bl[1]

    def acc(ea, eb):
        q = floor(Fraction(2 * dB * sign * (ea - eb), 1 << prog.S))
        return 1.0 if q >= 0 else X[max(q, -(O.XLEN - 1)) + O.XLEN - 1] / float(1 << 24)

    A = np.array([[acc(E[a], E[b]) for b in range(n)] for a in range(n)])
    # dist[p][a, b]: replica 0 in state a, replica 1 in b; p = 0: replica 0 hot
    dist = np.zeros((2, n, n))
    dist[0, 0, 0] = 1.0
    for t in range(prog.T):
        dist = np.stack([K[0].T @ dist[0] @ K[1], K[1].T @ dist[1] @ K[0]])
        if t % 2 == 0:
            a0 = A                  # p = 0: hot replica 0 (a) against cold replica 1 (b)
            a1 = A.T                # p = 1: hot replica 1 (b) against cold replica 0 (a)
            moved0, moved1 = dist[0] * a0, dist[1] * a1
            dist = np.stack([dist[0] - moved0 + moved1, dist[1] - moved1 + moved0])
    return dist[0].sum(axis=0) + dist[1].sum(axis=1)


def test_coldest_replica_follows_the_exact_joint_law():
    prob = G.tiny(4, 1, True, G.rng_for(951, 0), pmax=5, wmax=5)
    chains = 30000
    prog = _prog(prob, replicas=2 * chains, sweeps=6, beta=Fraction(3), p_q=2 * 256, pt_slots=2)
    assert prog.n_ext <= 7
    lq = [300]
    law = _exact_pt2_law(prog, lq)
    x, _, slot = O.pt_round(prog, lq, 0, 0, None, os.cpu_count())
    cold = x[slot == 1]
    assert len(cold) == chains
    counts = np.bincount(_state_codes(cold), minlength=len(law))
    assert _chi2_pvalue(counts, law) > 1e-4
    # the exchange with its sign reversed (hot and cold swapped in the rule)
    # gives another law, which these samples reject
    wrong = _exact_pt2_law(prog, lq, sign=-1)
    assert 0.5 * np.abs(wrong - law).sum() > 0.02
    assert _chi2_pvalue(counts, wrong) < 1e-6


def test_exchanges_happen_and_keep_a_permutation():
    prob = G.qkp(12, Fraction(1, 2), G.rng_for(952, 0))
    prog = _prog(prob, replicas=64, sweeps=40, beta=Fraction(8), eta=Fraction(2), pt_slots=16)
    x, g, slot = O.pt_round(prog, [0], 0, 0, None, 4)
    for c in range(4):
        s = slot[16 * c:16 * c + 16]
        assert sorted(s.tolist()) == list(range(16))
    assert (slot != np.arange(64) % 16).any()
    # residuals are those of the final states
    assert (g == O.residual(prog, x.astype(np.int64))).all()


def test_multiplier_step_averages_the_samples_only():
    prob = G.qkp(14, Fraction(1, 2), G.rng_for(953, 0))
    par = G.Params(replicas=32, sweeps=20, beta=Fraction(6), eta=Fraction(3), pt_slots=8)
    ref = O.saim(prob, par, 3, nthreads=4)
    prog = ref["program"]
    assert prog.samples == 4
    acc = [0]
    for k, e in enumerate(ref["rounds"]):
        sample = e["slot"] == 7
        assert sample.sum() == 4
        assert e["G"] == [int(v) for v in e["g"][sample].sum(axis=0)]
        # the step divides by the 4 samples, not the 32 replicas
        step = O.round_half_away(Fraction(1 << 32) * prog.eta * e["G"][0] / (4 * prog.s_g))
        acc = [max(-(prog.lq_max << 24), min(prog.lq_max << 24, acc[0] + step))]
        want = ref["rounds"][k + 1]["lq"] if k + 1 < len(ref["rounds"]) else ref["lq"]
        assert want == [O.round_half_away(Fraction(acc[0], 1 << 24))]


def test_settings_are_validated():
    prob = G.qkp(10, Fraction(1, 2), G.rng_for(954, 0))
    for bad in (dict(pt_slots=3), dict(pt_slots=2, replicas=63), dict(pt_slots=128, replicas=128)):
        kw = dict(replicas=64, sweeps=5, beta=Fraction(2))
        kw.update(bad)
        with pytest.raises(ValueError):
            _prog(prob, **kw)
    with pytest.raises(ValueError):
        _prog(G.mkp(10, 2, G.rng_for(954, 1)), replicas=64, sweeps=5, beta=Fraction(2), pt_slots=4)
