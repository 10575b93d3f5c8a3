"""GPU parity on seeded random shapes: sizes, densities, constraint counts,
replica and sweep counts, temperatures, steps and launch layouts drawn at
random (one generator per case), each run for two rounds against the oracle
bit for bit.  Shapes the library refuses are drawn again."""
from fractions import Fraction

import numpy as np
import pytest

from paper_2501_04971_amd import binding as B
from paper_2501_04971_amd import generators as G
from test_parity_gpu import assert_round_equal, say

from oracle import oracle as O

pytestmark = pytest.mark.gpu

BETAS = [Fraction(0), Fraction(1, 2), Fraction(5), Fraction(10), Fraction(50)]
ETAS = [Fraction(0), Fraction(1, 20), Fraction(1, 2), Fraction(20)]
DENS = [Fraction(1, 8), Fraction(1, 4), Fraction(1, 2), Fraction(3, 4), Fraction(1)]


def draw(case: int):
    rng = np.random.default_rng([97, case])
    while True:
        if case % 2 == 0:
            n = int(rng.integers(1, 321))
            prob = G.qkp(n, DENS[int(rng.integers(len(DENS)))], G.rng_for(970, case))
            alpha = Fraction(2)
        else:
            n, m = int(rng.integers(1, 201)), int(rng.integers(1, 33))
            prob = G.mkp(n, m, G.rng_for(971, case))
            alpha = Fraction(5)
        par = G.Params(replicas=int(rng.integers(1, 200)), sweeps=int(rng.integers(1, 26)),
                       beta=BETAS[int(rng.integers(len(BETAS)))], eta=ETAS[int(rng.integers(len(ETAS)))],
                       alpha=alpha, seed=int(rng.integers(1 << 31)), instance_id=case)
        layout = int(rng.integers(2))  # 0: the library's choice, 1: the plain layout
        try:
            B.pbit_plan(prob, par)
        except B.PbitError:
            continue
        return prob, par, layout


@pytest.mark.parametrize("case", range(48))
def test_random_shape(need_gpu, case):
    prob, par, layout = draw(case)
    say(f"[random] case {case}: kind {prob.kind} n={prob.n} m={prob.m} R={par.replicas} T={par.sweeps} "
        f"beta={par.beta} eta={par.eta} layout={'plain' if layout else 'default'}")
    rounds = 2
    ref = O.saim(prob, par, rounds, nthreads=8)
    inst = B.Instance(prob, par)
    try:
        if layout:
            inst.set_tiling(0, -1, 0)
        for k in range(rounds):
            lam = inst.get_lambda()
            inst.sample_round()
            out = inst.round_outputs()
            inst.update_lambda()
            out["lq"] = lam
            assert_round_equal(ref["program"], ref["rounds"][k], out, k)
        assert [int(v) for v in inst.get_lambda()] == ref["lq"]
        best = inst.best_feasible()
        if ref["best"] is None:
            assert best is None
        else:
            assert best is not None and best[0] == ref["best"][0]
            assert best[2] == ref["best"][1] and best[3] == ref["best"][2]
            assert (best[1] == ref["best"][3]).all()
    finally:
        inst.close()


def test_random_batch(need_gpu):
    """Twenty-four random members (the shapes above, other seeds) with round
    budgets of one to three, one persistent batch replayed as a graph: every
    member ends where the oracle's loop for it alone ends."""
    from test_batch_gpu import verify_final
    members = []
    for case in range(100, 124):
        prob, par, _ = draw(case)
        members.append((prob, par, 1 + case % 3))
    say(f"[random] batch of {len(members)} members")
    refs = [O.saim(p, q, K, nthreads=8) for p, q, K in members]
    batch = B.Batch([p for p, _, _ in members], [q for _, q, _ in members], rounds=[K for _, _, K in members])
    try:
        batch.run(4, use_graph=True)
        assert (batch.rounds_left() == 0).all()
        verify_final(batch, members, refs)
    finally:
        batch.close()


@pytest.mark.parametrize("case", range(16))
def test_random_tempering(need_gpu, case):
    """Parallel tempering on random quadratic shapes: chain length L of 2..64,
    R a multiple of L, random sweeps, temperatures, steps and layout."""
    rng = np.random.default_rng([98, case])
    n = int(rng.integers(1, 321))
    prob = G.qkp(n, DENS[int(rng.integers(len(DENS)))], G.rng_for(972, case))
    L = int(2 ** rng.integers(1, 7))
    par = G.Params(replicas=L * int(rng.integers(1, max(2, 200 // L + 1))), sweeps=int(rng.integers(1, 26)),
                   beta=BETAS[1 + int(rng.integers(len(BETAS) - 1))], eta=ETAS[int(rng.integers(len(ETAS)))],
                   seed=int(rng.integers(1 << 31)), instance_id=case, pt_slots=L)
    layout = int(rng.integers(2))
    say(f"[random] tempering case {case}: n={n} L={L} R={par.replicas} T={par.sweeps} beta={par.beta} "
        f"eta={par.eta} layout={'plain' if layout else 'default'}")
    rounds = 2
    ref = O.saim(prob, par, rounds, nthreads=8)
    inst = B.Instance(prob, par)
    try:
        if layout:
            inst.set_tiling(0, -1, 0)
        for k in range(rounds):
            assert [int(v) for v in inst.get_lambda()] == ref["rounds"][k]["lq"], f"round {k}: multipliers"
            inst.sample_round()
            out = inst.round_outputs()
            inst.update_lambda()
            e = ref["rounds"][k]
            x = B.unpack_bits(out["x_bits"], ref["program"].n_ext)
            bad = np.nonzero((x != e["x"]).any(axis=1))[0]
            assert bad.size == 0, f"round {k}: {bad.size} replicas differ, first {bad[:4]}"
            assert (out["g"] == e["g"]).all(), f"round {k}: residuals"
            assert (out["slot"] == e["slot"]).all(), f"round {k}: ladder positions"
            assert (out["profit"] == e["profit"]).all()
            assert (out["feasible"].astype(bool) == e["feasible_mask"]).all()
            assert [int(v) for v in out["G"]] == e["G"], f"round {k}: residual sums of the samples"
        assert [int(v) for v in inst.get_lambda()] == ref["lq"]
        best = inst.best_feasible()
        if ref["best"] is None:
            assert best is None
        else:
            assert best is not None and best[0] == ref["best"][0] and best[2:] == (ref["best"][1], ref["best"][2])
    finally:
        inst.close()
