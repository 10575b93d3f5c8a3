"""Several instances on streams of their own, every round of every instance
queued before any result is read: each instance's last round, multipliers
and best record equal the oracle's, as when it runs alone (instances share no
device state; one of them uses the library's allocation-free workspace, one
runs parallel tempering)."""
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


def test_instances_on_streams_of_their_own(need_gpu):
    import torch
    cases = [
        ("QKP n=70", G.qkp(70, Fraction(1, 2), G.rng_for(960, 0)),
         G.Params(replicas=128, sweeps=40, beta=Fraction(10), eta=Fraction(200)), False),
        ("MKP n=60 m=5 (static workspace)", G.mkp(60, 5, G.rng_for(960, 1)),
         G.Params(replicas=100, sweeps=30, beta=Fraction(50), eta=Fraction(1, 2), alpha=Fraction(5)), True),
        ("QKP n=150", G.qkp(150, Fraction(1, 4), G.rng_for(960, 2)),
         G.Params(replicas=64, sweeps=30, beta=Fraction(10), eta=Fraction(1500), seed=7), False),
        ("QKP n=70, tempering L=4", G.qkp(70, Fraction(1, 2), G.rng_for(960, 0)),
         G.Params(replicas=128, sweeps=40, beta=Fraction(10), eta=Fraction(200), pt_slots=4), False),
    ]
    rounds = 4  # (steps large enough that every instance has a feasible sample by then)
    refs = [O.saim(p, q, rounds, nthreads=8) for _, p, q, _ in cases]
    assert all(r["best"] is not None for r in refs)
    streams = [torch.cuda.Stream() for _ in cases]
    insts = []
    try:
        for (label, p, q, static), st in zip(cases, streams):
            say(f"[streams] create {label}")
            with torch.cuda.stream(st):
                insts.append(B.Instance(p, q, stream=st, static_workspace=static))
        say(f"[streams] {rounds} rounds queued on {len(insts)} streams")
        for _ in range(rounds):
            for inst in insts:
                inst.sample_round()
                inst.update_lambda()
        torch.cuda.synchronize()
        for (label, _, _, _), inst, ref in zip(cases, insts, refs):
            say(f"[streams] check {label}")
            e = ref["rounds"][-1]
            out = inst.round_outputs()
            x = B.unpack_bits(out["x_bits"], ref["program"].n_ext)
            bad = np.nonzero((x != e["x"]).any(axis=1))[0]
            assert bad.size == 0, f"{label}: {bad.size} replicas differ in the last round, first {bad[:4]}"
            assert (out["g"] == e["g"]).all(), f"{label}: residuals"
            assert (out["profit"] == e["profit"]).all(), f"{label}: profits"
            assert (out["feasible"].astype(bool) == e["feasible_mask"]).all(), f"{label}: feasibility"
            assert [int(v) for v in out["G"]] == e["G"], f"{label}: residual sums"
            assert [int(v) for v in inst.get_lambda()] == ref["lq"], f"{label}: multipliers"
            best = inst.best_feasible()
            if ref["best"] is None:
                assert best is None, label
            else:
                assert best is not None and best[0] == ref["best"][0], f"{label}: best profit"
                assert best[2:] == (ref["best"][1], ref["best"][2]), f"{label}: best round and replica"
                assert (best[1] == ref["best"][3]).all(), f"{label}: best state"
    finally:
        for inst in insts:
            inst.close()
