"""Autotuner: shape keys, candidate sets and the JSON cache on the host; on the
GPU, tuning picks a layout whose results are the oracle's."""
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2501_04971_amd import autotune as A
from paper_2501_04971_amd import binding as B
from paper_2501_04971_amd import generators as G


def test_keys_candidates_and_cache(tmp_path):
    q = G.qkp(90, Fraction(1, 2), G.rng_for(980, 0))
    m = G.mkp(120, 7, G.rng_for(980, 1))
    par = G.Params(replicas=300, sweeps=10)
    iq, im = B.pbit_plan(q, par), B.pbit_plan(m, par)
    assert iq.n_pad == (iq.n_ext + 31) // 32 * 32
    assert A.shape_key(iq, 300) == f"v0-n{iq.n_pad}-m1-r512"
    assert A.shape_key(im, 300).startswith("v1-n") and A.shape_key(im, 300).endswith("-m7-r512")
    assert A.candidates(iq) == [(1, -1, 0), (4, -1, 0), (4, -1, 1), (4, -1, 2)]
    assert len(A.candidates(im)) == 9
    path = str(tmp_path / "t.json")
    assert A.load_cache(path) == {}
    A.save_cache({"k": {"waves_per_block": 4, "lds_resident": -1}}, path)
    assert A.load_cache(path)["k"]["waves_per_block"] == 4


@pytest.mark.gpu
def test_tuned_layout_is_used_and_exact(need_gpu, tmp_path):
    from oracle import oracle as O
    path = str(tmp_path / "tiling.json")
    prob = G.mkp(100, 5, G.rng_for(981, 0))
    par = G.Params(replicas=200, sweeps=20, beta=Fraction(50), eta=Fraction(1, 2), alpha=Fraction(5))
    entry = A.tune_instance(prob, par, probe_sweeps=10, reps=1, path=path)
    assert len(entry["probe_ms"]) == 9
    inst = B.Instance(prob, par)
    got = A.apply(inst, prob, par, tune_missing=False, path=path)
    assert got == entry
    inst.sample_round()
    out = inst.round_outputs()
    inst.close()
    ref = O.saim(prob, par, 1, nthreads=8)["rounds"][0]
    assert (B.unpack_bits(out["x_bits"], ref["x"].shape[1]) == ref["x"]).all()
    assert (out["g"] == ref["g"]).all()


def test_batch_key_and_candidates():
    members = [G.workload(3, i) for i in range(4)]
    probs, pars = [p for p, _, _ in members], [q for _, q, _ in members]
    k = A.batch_key(probs, pars)
    assert k.startswith("batch-4-") and k == A.batch_key(probs[::-1], pars[::-1])  # order-free
    assert k != A.batch_key(probs[:3], pars[:3])
    cands = A.batch_candidates()
    assert {c["split_percent"] for c in cands} == {0, 150, 200, 300}
    probe = A.probe_params(pars, 80)
    # one common factor: the members keep their sweep ratio
    assert [q.sweeps for q in probe] == [q.sweeps // (max(p.sweeps for p in pars) // 80) for q in pars]


@pytest.mark.gpu
def test_tuned_batch_layout_is_used_and_exact(need_gpu, tmp_path):
    """A tuned mixed batch is re-created with the timed layout and its round is
    the oracle's, member by member."""
    from oracle import oracle as O
    path = str(tmp_path / "tiling.json")
    small = []
    for i in range(6):
        p, q, _ = G.workload(3, i)
        small.append((p, G.Params(replicas=64, sweeps=q.sweeps // 50, beta=q.beta, eta=q.eta, alpha=q.alpha,
                                  instance_id=q.instance_id)))
    probs, pars = [p for p, _ in small], [q for _, q in small]
    entry = A.tune_batch(probs, pars, probe_sweeps=10, reps=1, path=path)
    assert len(entry["probe_ms"]) >= 4
    lay = A.batch_layout(probs, pars, tune_missing=False, path=path)
    assert lay == entry["layout"]
    b = B.Batch(probs, pars, rounds=[1] * len(small), layout=lay)
    used = b.layout()
    assert used["split_percent"] == lay["split_percent"]
    assert lay["blocks_linear"] == 0 or used["blocks_linear"] <= lay["blocks_linear"]
    b.run(1, use_graph=True)
    for i, (p, q) in enumerate(small):
        out = b.members[i].round_outputs()
        ref = O.saim(p, q, 1, nthreads=8)["rounds"][0]
        x = B.unpack_bits(out["x_bits"], ref["x"].shape[1])
        assert (x == ref["x"]).all(), f"member {i}"
        assert (out["g"][:, :p.m] == ref["g"]).all()
    b.close()
