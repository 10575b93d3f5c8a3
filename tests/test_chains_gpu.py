"""Independent chains with their own multipliers: R single-chain runs of
Algorithm 1 (lambda stepped after every run of that chain alone) as R members
of one batch, each checked round by round against the oracle's Algorithm 1
with one replica.  This is the paper's loop itself (one IM run per iteration,
Algorithm 1), run many times side by side, as opposed to the replica-mean
multiplier step of a single instance."""
import sys
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_04971_amd import binding as B
from paper_2501_04971_amd import generators as G

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kind", ["qkp", "mkp"])
def test_independent_chains_follow_algorithm_1(need_gpu, kind):
    if kind == "qkp":
        prob = G.qkp(50, Fraction(1, 2), G.rng_for(993, 0))
        base = dict(sweeps=60, beta=Fraction(10), eta=Fraction(20), alpha=Fraction(2))
    else:
        prob = G.mkp(60, 5, G.rng_for(993, 1))
        base = dict(sweeps=40, beta=Fraction(50), eta=Fraction(1), alpha=Fraction(5))
    chains, rounds = 8, 12
    pars = [G.Params(replicas=1, instance_id=c, **base) for c in range(chains)]
    say(f"[chains] {kind}: {chains} chains x {rounds} rounds")
    batch = B.Batch([prob] * chains, pars, rounds=[rounds] * chains)
    snap = torch.empty((rounds, chains * B.SNAPSHOT_BYTES), dtype=torch.uint8, device="cuda")
    for k in range(rounds):
        batch.run(1, use_graph=True)
        batch.snapshot(snap[k])
    torch.cuda.synchronize()
    raw = snap.cpu().numpy()
    finals = [m.get_lambda() for m in batch.members]
    bests = [m.best_feasible() for m in batch.members]
    batch.close()
    recs = [B.decode_snapshot(raw[k], chains) for k in range(rounds)]
    distinct = set()
    for c in range(chains):
        ref = O.saim(prob, pars[c], rounds, nthreads=1)
        for k in range(rounds):
            # multipliers after round k's step are those in force at round k + 1
            want = ref["rounds"][k + 1]["lq"] if k + 1 < rounds else ref["lq"]
            assert [int(v) for v in recs[k]["lambda_q"][c, :prob.m]] == want, f"chain {c} round {k}"
            assert int(recs[k]["feasible_last"][c]) == ref["rounds"][k]["feasible"]
        assert [int(v) for v in finals[c]] == ref["lq"]
        if ref["best"] is None:
            assert bests[c] is None
        else:
            assert bests[c][0] == ref["best"][0] and bests[c][2] == ref["best"][1]
        distinct.add(tuple(ref["lq"]))
    assert len(distinct) > 1  # the chains draw different noise and end at different multipliers
