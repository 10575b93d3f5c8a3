"""The exact-optimum reference (branch and bound) against brute-force
enumeration of every assignment (the OPT of Sec. IV-A, Eq. accuracy)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from paper_2501_04971_amd import exact as E
from paper_2501_04971_amd import generators as G

PAR = G.Params(replicas=8, sweeps=10, beta=Fraction(5), eta=Fraction(1))


def brute_opt(prob):
    return brute.opt_max(O.build_program(prob, PAR))


@pytest.mark.parametrize("seed", range(12))
def test_matches_enumeration_on_tiny_instances(seed):
    rng = G.rng_for(4000, seed)
    quadratic = seed % 2 == 0
    n = int(rng.integers(4, 15))
    m = 1 if quadratic else int(rng.integers(1, 4))
    prob = G.tiny(n, m, quadratic, rng)
    want, _ = brute_opt(prob)
    got = E.solve(prob, time_limit=60)
    assert got.proven
    assert got.profit == want
    assert E.feasible(prob, got.x) and E.profit_of(prob, got.x) == want


def test_negative_pair_profits():
    """Pairs that lose value need the lower linking rows y >= x_i + x_j - 1."""
    rng = G.rng_for(4001, 0)
    for trial in range(6):
        n = 10
        vals = rng.integers(-9, 10, size=(n, n))
        upper = np.triu(vals)
        p = (upper + np.triu(upper, 1).T).astype(np.int32)
        a = rng.integers(1, 10, size=(1, n)).astype(np.int32)
        b = np.array([int(a.sum()) // 2], dtype=np.int64)
        prob = G.Problem(G.KIND_QKP, p, a, b, Fraction(1, 2), "neg")
        # profit of the original bits by enumeration (no slack needed here)
        xs = brute.all_states(n)
        prof = np.array([E.profit_of(prob, x) for x in xs])
        feas = (xs @ a[0].astype(np.int64)) <= b[0]
        want = int(prof[feas].max())
        got = E.solve(prob, time_limit=60)
        assert got.proven and got.profit == want, trial


def test_profit_of_counts_each_pair_once():
    p = np.array([[3, 5, 0], [5, 2, 7], [0, 7, 1]], dtype=np.int32)
    prob = G.Problem(G.KIND_QKP, p, np.ones((1, 3), dtype=np.int32), np.array([3], dtype=np.int64))
    assert E.profit_of(prob, np.array([1, 1, 1])) == 3 + 2 + 1 + 5 + 7
    assert E.profit_of(prob, np.array([1, 0, 1])) == 3 + 1


def test_mid_size_qkp_is_proven_and_dominates_the_sampler_record():
    """N = 40: proven optimum, feasible, and no smaller than any feasible
    assignment found by the oracle's own sampler on the same instance."""
    prob = G.qkp(40, Fraction(1, 2), G.rng_for(4002, 0))
    got = E.solve(prob, time_limit=120)
    assert got.proven and E.feasible(prob, got.x)
    ref = O.saim(prob, G.Params(replicas=16, sweeps=200, beta=Fraction(10), eta=Fraction(20)), 8, nthreads=4)
    if ref["best"] is not None:
        assert ref["best"][0] <= got.profit
