"""Parallel tempering as the machine inside Algorithm 1 on the GPU, against the
oracle bit for bit: every replica's final state and residual, its ladder
position, the chains' samples' residual sums, the multipliers each round and
the best record, in the split layout (the default: producers hand over each
draw's table position, the visiting wave compares it with its own field's
index at its lane's temperature) and in the plain one."""
import sys
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_04971_amd import binding as B
from paper_2501_04971_amd import generators as G

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,L,R,wpb,split", [(40, 4, 64, 0, -1), (70, 16, 128, 1, -1), (100, 64, 128, 0, -1),
                                             (33, 2, 96, 0, -1), (300, 32, 128, 0, -1), (40, 4, 64, 1, 0),
                                             (100, 64, 128, 4, 0)])
def test_parallel_tempering_matches_oracle(need_gpu, n, L, R, wpb, split):
    prob = G.qkp(n, Fraction(1, 2), G.rng_for(994, n))
    par = G.Params(replicas=R, sweeps=40, beta=Fraction(10), eta=Fraction(20), pt_slots=L)
    rounds = 3
    say(f"[pt] n={n} L={L} R={R} wpb={wpb} split={split}")
    ref = O.saim(prob, par, rounds, nthreads=8)
    prog = ref["program"]
    inst = B.Instance(prob, par)
    if wpb or split != -1:
        inst.set_tiling(wpb, -1, split)
    for k in range(rounds):
        assert [int(v) for v in inst.get_lambda()] == ref["rounds"][k]["lq"], f"round {k}: multipliers"
        inst.sample_round()
        out = inst.round_outputs()
        inst.update_lambda()
        e = ref["rounds"][k]
        x = B.unpack_bits(out["x_bits"], prog.n_ext)
        bad = np.nonzero((x != e["x"]).any(axis=1))[0]
        assert bad.size == 0, f"round {k}: {bad.size} replicas differ, first {bad[:4]}"
        assert (out["g"] == e["g"]).all(), f"round {k}: residuals"
        assert (out["slot"] == e["slot"]).all(), f"round {k}: ladder positions"
        assert (out["profit"] == e["profit"]).all() and (out["feasible"].astype(bool) == e["feasible_mask"]).all()
        assert [int(v) for v in out["G"]] == e["G"], f"round {k}: residual sums of the samples"
    assert [int(v) for v in inst.get_lambda()] == ref["lq"]
    best = inst.best_feasible()
    inst.close()
    if ref["best"] is None:
        assert best is None
    else:
        assert best is not None and best[0] == ref["best"][0] and best[2:] == (ref["best"][1], ref["best"][2])
    # exchanges happened
    assert any((e["slot"] != np.arange(R) % L).any() for e in ref["rounds"])
