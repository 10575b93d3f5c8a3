"""Host side of the learned-lambda_0 path: the library's feature packing against
the oracle's features, bit for bit after bfloat16 rounding."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import lambda_net as N
from oracle import oracle as O
from paper_2501_04971_amd import binding as B
from paper_2501_04971_amd import generators as G


def bits(v):
    return (N.bf16(v).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def members():
    out = [G.workload(3, i)[:2] for i in range(4)]
    out.append((G.qkp(37, Fraction(1, 2), G.rng_for(960, 0)), G.Params(replicas=64, sweeps=10)))
    out.append((G.mkp(70, 3, G.rng_for(960, 1)), G.Params(replicas=64, sweeps=10, beta=Fraction(50),
                                                              alpha=Fraction(5))))
    return out


@pytest.fixture(scope="module")
def lib():
    return B.lib()


def test_pack_matches_oracle_features(lib):
    ms = members()
    pk = B.pbit_net_pack([p for p, _ in ms], [q for _, q in ms])
    s = 0
    for i, (prob, par) in enumerate(ms):
        prog = O.build_program(prob, par)
        for f in N.instance_features(prob, par, prog.n_ext, prog.pq, member=i):
            r0, n = pk["set_rows"][s], pk["set_n"][s]
            assert r0 % 32 == 0 and n == prob.n
            assert pk["set_rows"][s + 1] - r0 == (prob.n + 31) // 32 * 32
            assert (pk["x"][r0:r0 + n] == bits(f.X)).all(), f"set {s}: features differ"
            assert not pk["x"][r0 + n:pk["set_rows"][s + 1]].any()
            assert (pk["ctx"][s, :9] == bits(f.ctx)).all() and not pk["ctx"][s, 9:].any()
            assert pk["scale"][s] == f.scale
            assert pk["dest"][s] == i * 32 + f.k
            s += 1
    assert s == pk["sets"] and pk["set_rows"][s] == pk["rows"]


def test_layout_constants(lib):
    assert B.pbit_net_param_count() == N.N_PARAMS == 37377
    assert B.pbit_net_workspace_bytes(0, 32) == 0
    assert B.pbit_net_workspace_bytes(3, 40) == 0
    assert B.pbit_net_workspace_bytes(3, 96) > 0
