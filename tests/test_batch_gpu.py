"""GPU parity of the batched path: a batch member must produce exactly what the
oracle's loop produces for that instance alone (Tables 2-5 solve every
instance independently), whatever the other members, the queue order, the
persistent grid size or the graph replay."""
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_04971_amd import binding as B
from paper_2501_04971_amd import generators as G

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mixed_members():
    """Uneven sizes of both kinds: 1..11 site blocks, constraint counts with and
    without a batch body of their own (7 pads to 8, 12 to 16), replica counts
    that leave partial tiles, per-member round budgets."""
    out = []
    specs = [("q", 20, Fraction(1), 64, 3), ("q", 97, Fraction(3, 4), 300, 2),
             ("q", 200, Fraction(1, 4), 256, 4), ("q", 330, Fraction(1, 2), 70, 1),
             ("m", 40, 1, 64, 3), ("m", 60, 7, 130, 4), ("m", 100, 30, 256, 2),
             ("m", 120, 12, 64, 3), ("m", 250, 10, 100, 2)]
    for i, (kind, n, x, R, K) in enumerate(specs):
        if kind == "q":
            prob = G.qkp(n, x, G.rng_for(930, i))
            par = G.Params(replicas=R, sweeps=30 + 7 * i, beta=Fraction(5), eta=Fraction(20),
                           instance_id=i)
        else:
            prob = G.mkp(n, x, G.rng_for(931, i))
            par = G.Params(replicas=R, sweeps=25 + 5 * i, beta=Fraction(50), eta=Fraction(1, 2),
                           alpha=Fraction(5), instance_id=i)
        out.append((prob, par, K))
    return out


def check_member(member, prob, ref_round, k, m_orig):
    got = member.round_outputs()
    prog = None
    x = B.unpack_bits(got["x_bits"], ref_round["x"].shape[1])
    bad = np.nonzero((x != ref_round["x"]).any(axis=1))[0]
    assert bad.size == 0, f"round {k}: {bad.size} replicas differ (first {bad[0]})"
    assert (got["g"][:, :m_orig] == ref_round["g"]).all(), f"round {k}: residuals differ"
    assert (got["g"][:, m_orig:] == 0).all(), "padding constraints must stay empty"
    assert (got["profit"] == ref_round["profit"]).all(), f"round {k}: profits differ"
    assert (got["feasible"].astype(bool) == ref_round["feasible_mask"]).all()
    assert [int(v) for v in got["G"][:m_orig]] == ref_round["G"]
    return got, prog


@pytest.fixture(scope="module")
def mixed_refs():
    members = mixed_members()
    refs = []
    for prob, par, K in members:
        refs.append(O.saim(prob, par, K, nthreads=NTHREADS))
    return members, refs


def verify_final(batch, members, refs):
    for i, ((prob, par, K), ref) in enumerate(zip(members, refs)):
        mem = batch.members[i]
        lam = mem.get_lambda()
        assert [int(v) for v in lam[:prob.m]] == ref["lq"], f"member {i}: final multipliers differ"
        assert (lam[prob.m:] == 0).all()
        best = mem.best_feasible()
        if ref["best"] is None:
            assert best is None, f"member {i}"
        else:
            assert best is not None, f"member {i}: best feasible missing"
            assert (best[0], best[2], best[3]) == ref["best"][:3], f"member {i}: best differs"
            assert (best[1] == ref["best"][3]).all()
        # the last round a member ran is its budget's last round
        check_member(mem, prob, ref["rounds"][K - 1], K - 1, prob.m)
        assert mem.round_outputs()["round"] == K


@pytest.mark.parametrize("blocks", [0, 3])
def test_batch_direct_launches(need_gpu, mixed_refs, blocks):
    """Direct launches; blocks=3 forces every workgroup through many queue items."""
    members, refs = mixed_refs
    say(f"[batch] direct launches, {len(members)} members, blocks={blocks}")
    batch = B.Batch([p for p, _, _ in members], [q for _, q, _ in members],
                    rounds=[K for _, _, K in members], blocks=blocks)
    items, nblk, lds = batch.shape()
    say(f"[batch] items={items} blocks={nblk} lds={lds}")
    Kmax = max(K for _, _, K in members)
    batch.run(Kmax + 2, use_graph=False)  # extra rounds: budgets stop every member
    left = batch.rounds_left()
    assert (left == 0).all()
    verify_final(batch, members, refs)
    batch.close()


def test_batch_graph_replays(need_gpu, mixed_refs):
    """Graph replays one round at a time with host reads in between; every
    replay is checked against the oracle's round for every member still running."""
    import torch
    members, refs = mixed_refs
    say(f"[batch] graph replays, {len(members)} members")
    batch = B.Batch([p for p, _, _ in members], [q for _, q, _ in members],
                    rounds=[K for _, _, K in members])
    Kmax = max(K for _, _, K in members)
    for k in range(Kmax):
        batch.run(1, use_graph=True)
        torch.cuda.synchronize()
        left = batch.rounds_left()
        for i, ((prob, par, K), ref) in enumerate(zip(members, refs)):
            assert left[i] == max(0, K - k - 1)
            if k < K:
                check_member(batch.members[i], prob, ref["rounds"][k], k, prob.m)
                lam = batch.members[i].get_lambda()
                nxt = ref["rounds"][k + 1]["lq"] if k + 1 < K else ref["lq"]
                assert [int(v) for v in lam[:prob.m]] == nxt, f"member {i} round {k}: multipliers"
    verify_final(batch, members, refs)
    batch.close()


def test_batch_member_set_lambda(need_gpu):
    """A member started from given multipliers (the learned-start path) matches
    the oracle started there; its neighbours are unaffected."""
    members = mixed_members()[4:7]
    lq0 = [[900], [500, -300, 0, 40, 7, 1, 2], [0] * 30]
    refs = [O.saim(p, q, K, lq0=l, nthreads=NTHREADS) for (p, q, K), l in zip(members, lq0)]
    batch = B.Batch([p for p, _, _ in members], [q for _, q, _ in members],
                    rounds=[K for _, _, K in members])
    for mem, (p, _, _), l in zip(batch.members, members, lq0):
        padded = list(l) + [0] * (mem.info.m - p.m)
        mem.set_lambda(padded)
    batch.run(max(K for _, _, K in members), use_graph=True)
    verify_final(batch, members, refs)
    batch.close()


def test_batch_workload3_sampled(need_gpu):
    """The full mixed workload (512 members: 256 QKP N in U{100..300}, 256 MKP N in
    {100,250,500} x M in {5,10,30}, 256 replicas each) for two graph rounds.  For
    sampled members, sampled replicas of round 0 (lambda = 0) and of round 1
    (under the multipliers the first step gave, checked against the oracle's
    step) are replayed by the oracle."""
    import torch
    members = [G.workload(3, i) for i in range(512)]
    batch = B.Batch([p for p, _, _ in members], [q for _, q, _ in members],
                    rounds=[K for _, _, K in members])
    items, nblk, lds = batch.shape()
    say(f"[batch] workload 3: items={items} blocks={nblk} lds={lds}")
    rng = np.random.default_rng(5)
    # 7, 21 and 51 are MKP members that take the 64-bit dot kernels (N=250 M=30, N=500 M=30, N=500 M=10)
    picks = [0, 1, 2, 3, 7, 21, 51] + [int(v) for v in rng.choice(np.arange(4, 512), 6, replace=False)]
    reps = {i: sorted({0, 255, int(rng.integers(1, 255))}) for i in picks}
    progs = {i: O.build_program(members[i][0], members[i][1]) for i in picks}
    acc = {i: [0] * members[i][0].m for i in picks}
    lq = {i: [0] * members[i][0].m for i in picks}
    moved = set()
    for k in range(2):
        batch.run(1, use_graph=True)
        torch.cuda.synchronize()
        for i in picks:
            prob, par, K = members[i]
            prog = progs[i]
            if k == 1 and any(v != 0 for v in lq[i]):
                moved.add(i)
            got = batch.members[i].round_outputs()
            lam = batch.members[i].get_lambda()
            for r in reps[i]:
                say(f"[batch] round {k} member {i} {prob.name} replica {r}")
                x, g = O.sa_round(prog, lq[i], k, r, 1, 1)
                xb = B.unpack_bits(got["x_bits"][r:r + 1], prog.n_ext)
                assert (xb[0] == x[0]).all(), f"round {k} member {i} replica {r}: state differs"
                assert (got["g"][r, :prob.m] == g[0]).all()
            # the residual sums are the sums of the per-replica residuals
            assert (got["G"] == got["g"].astype(np.int64).sum(axis=0)).all()
            assert got["round"] == k + 1
            acc[i], lq[i] = O.lambda_step(prog, acc[i], [int(v) for v in got["G"][:prob.m]], k=k)
            assert [int(v) for v in lam[:prob.m]] == lq[i], f"round {k} member {i}: multipliers"
    assert len(moved) >= 3, moved  # round 1 ran at lambda != 0 (the QKP members)
    batch.close()
