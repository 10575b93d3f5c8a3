"""The allocation-free instance (pbit_create_instance_static) against the
instance on a caller workspace (pbit_create_instance), bit for bit.

Two static instances are made one after the other on the same device (the
second smaller than the first, so it runs on what the first left in the
static array); each runs three rounds of Algorithm 1 with the multipliers
moving and is compared round by round, together with the best record, with
the same problem run on a caller-owned workspace."""
import sys
from fractions import Fraction

import numpy as np
import pytest

from paper_2501_04971_amd import binding as B
from paper_2501_04971_amd import generators as G

pytestmark = pytest.mark.gpu

ROUNDS = 3


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(prob, par, static):
    inst = B.Instance(prob, par, static_workspace=static)
    log = []
    for _ in range(ROUNDS):
        inst.sample_round()
        log.append(inst.round_outputs())
        inst.update_lambda()
    best = inst.best_feasible()
    lam = inst.get_lambda()
    inst.close()
    return log, best, lam


def assert_same(a, b):
    log_a, best_a, lam_a = a
    log_b, best_b, lam_b = b
    for k, (ra, rb) in enumerate(zip(log_a, log_b)):
        for key in ("x_bits", "g", "profit", "feasible", "G", "lambda_q"):
            assert np.array_equal(ra[key], rb[key]), f"round {k}: {key} differs"
        assert ra["round"] == rb["round"] == k + 1
        assert ra["lambda_saturated"] == rb["lambda_saturated"]
    assert np.array_equal(lam_a, lam_b)
    assert (best_a is None) == (best_b is None)
    if best_a is not None:
        assert best_a[0] == best_b[0] and best_a[2:] == best_b[2:]
        assert np.array_equal(best_a[1], best_b[1])


def test_static_instances_match_caller_workspace(need_gpu):
    import torch
    first = (G.mkp(100, 5, G.rng_for(991, 0)),
             G.Params(replicas=256, sweeps=60, beta=Fraction(50), eta=Fraction(2), alpha=Fraction(5)))
    second = (G.qkp(40, Fraction(1, 2), G.rng_for(991, 1)),
              G.Params(replicas=64, sweeps=40, beta=Fraction(10), eta=Fraction(20)))
    sizes = [B.pbit_workspace_bytes(p, q) for p, q in (first, second)]
    assert sizes[1] < sizes[0] <= B.pbit_static_workspace_bytes()
    for label, (prob, par) in (("first (MKP n=100 m=5)", first), ("second (QKP n=40)", second)):
        say(f"[no-alloc] {label}: caller workspace")
        ref = run(prob, par, static=False)
        say(f"[no-alloc] {label}: static workspace")
        got = run(prob, par, static=True)
        torch.cuda.synchronize()
        assert_same(ref, got)


def test_static_workspace_is_exclusive_and_bounded(need_gpu):
    prob = G.qkp(30, Fraction(1, 2), G.rng_for(991, 2))
    par = G.Params(replicas=64, sweeps=10, beta=Fraction(5), eta=Fraction(1))
    say("[no-alloc] exclusivity and size bound")
    held = B.Instance(prob, par, static_workspace=True)
    with pytest.raises(B.PbitError) as err:
        B.pbit_create_instance_static(prob, par)
    assert err.value.status == -5  # PBIT_ESTATE while the first one is live
    held.close()
    again = B.Instance(prob, par, static_workspace=True)  # released by destroy
    again.close()
    big = G.Params(replicas=1 << 20, sweeps=10, beta=Fraction(5), eta=Fraction(1))
    assert B.pbit_workspace_bytes(prob, big) > B.pbit_static_workspace_bytes()
    with pytest.raises(B.PbitError) as err:
        B.pbit_create_instance_static(prob, big)
    assert err.value.status == -3  # PBIT_EWORKSPACE
