"""Host-only checks of the C ABI: the library loads, exports every declared
entry point, compiles instances to the same integers as the oracle, and
rejects malformed input with the documented status codes.  No GPU calls."""
import ctypes
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_04971_amd import binding as B
from paper_2501_04971_amd import build as BUILD
from paper_2501_04971_amd import generators as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(BUILD.LIB):
        BUILD.build()
    return B.lib()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pbit.h")).read()
    return sorted(set(re.findall(r"\b(pbit_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
        assert name in B.EXPORTS, name


def _cases():
    out = [G.workload(0, 0), G.workload(0, 5), G.workload(1, 0), G.workload(2, 0)]
    out += [G.workload(3, i) for i in range(6)]
    prob = G.tiny(7, 2, False, G.rng_for(910, 0))
    out.append((prob, G.Params(replicas=10, sweeps=7, beta=Fraction(3, 2), p_q=300), 1))
    prob = G.tiny(9, 1, True, G.rng_for(910, 1))
    out.append((prob, G.Params(replicas=3, sweeps=1, beta=Fraction(2), fixed_beta=True), 1))
    return out


@pytest.mark.parametrize("case", range(12))
def test_plan_matches_oracle_program(lib, case):
    prob, par, _ = _cases()[case]
    info = B.pbit_plan(prob, par)
    prog = O.build_program(prob, par)
    assert info.n_ext == prog.n_ext
    assert info.s_f == prog.s_f and info.s_g == prog.s_g
    assert info.p_q == prog.pq
    assert info.shift == prog.S
    assert info.lq_max == prog.lq_max
    assert info.workspace_bytes == B.pbit_workspace_bytes(prob, par) > 0
    assert info.words == (prog.n_ext + 31) // 32
    assert info.variant == (0 if prob.kind == G.KIND_QKP else info.variant)


def test_theta_table_matches_oracle(lib):
    assert B.pbit_theta_table().tolist() == list(O.theta_table())
    assert B.pbit_exchange_table().tolist() == list(O.exchange_table())


def _expect(status, prob, par):
    with pytest.raises(B.PbitError) as ei:
        B.pbit_plan(prob, par)
    assert ei.value.status == status
    assert B.pbit_workspace_bytes(prob, par) == 0


def test_error_codes(lib):
    prob, par, _ = G.workload(0, 0)
    bad = G.Problem(7, prob.profit, prob.weight, prob.capacity, prob.density)
    _expect(B.PBIT_EINVAL, bad, par)
    asym = np.array(prob.profit)
    asym[0, 1] += 1
    _expect(B.PBIT_EINVAL, G.Problem(G.KIND_QKP, asym, prob.weight, prob.capacity, prob.density), par)
    neg = np.array(prob.weight)
    neg[0, 3] = -1
    _expect(B.PBIT_EINVAL, G.Problem(G.KIND_QKP, prob.profit, neg, prob.capacity, prob.density), par)
    big = np.array(prob.profit)
    big[2, 2] = 200
    _expect(B.PBIT_ERANGE, G.Problem(G.KIND_QKP, big, prob.weight, prob.capacity, prob.density), par)
    two = G.Problem(G.KIND_QKP, prob.profit, np.vstack([prob.weight, prob.weight]),
                    np.concatenate([prob.capacity, prob.capacity]), prob.density)
    _expect(B.PBIT_ERANGE, two, par)
    wide = G.qkp(345, Fraction(1, 2), G.rng_for(911, 0))
    _expect(B.PBIT_ERANGE, wide, par)
    _expect(B.PBIT_EINVAL, prob, G.Params(replicas=0))
    _expect(B.PBIT_EINVAL, prob, G.Params(sweeps=0))
    _expect(B.PBIT_EINVAL, prob, G.Params(eta=Fraction(-1)))


def test_null_workspace_is_rejected_before_any_device_call(lib):
    prob, par, _ = G.workload(0, 0)
    mp = B._Marshalled(prob, par)
    h = ctypes.c_void_p()
    st = lib.pbit_create_instance(ctypes.byref(mp.problem), ctypes.byref(mp.params), None, 0, None,
                                  ctypes.byref(h))
    assert st == B.PBIT_EWORKSPACE and h.value is None
    assert lib.pbit_sample_round(None, None) == B.PBIT_EINVAL
    assert b"null instance" in lib.pbit_last_error()


def test_batch_sizes_and_member_errors(lib):
    """Batch workspace covers every member's own workspace plus the queue; a bad
    member is named in the message; constraint counts without a batch body are
    padded (their plan is the padded one, with no extra slack bits)."""
    members = [G.workload(3, i) for i in range(6)]
    probs = [p for p, _, _ in members]
    pars = [q for _, q, _ in members]
    total = B.pbit_batch_workspace_bytes(probs, pars)
    assert total > sum(B.pbit_workspace_bytes(p, q) for p, q in zip(probs, pars))
    mk = G.mkp(60, 7, G.rng_for(940, 0))
    par = G.Params(replicas=64, sweeps=10, beta=Fraction(50), alpha=Fraction(5))
    assert B.pbit_batch_workspace_bytes([mk], [par]) >= B.pbit_workspace_bytes(mk, par)
    padded = G.Problem(G.KIND_MKP, mk.profit, np.vstack([mk.weight, np.zeros((1, 60), np.int64)]),
                       np.concatenate([mk.capacity, [0]]), mk.density)
    assert B.pbit_plan(padded, par).n_ext == B.pbit_plan(mk, par).n_ext
    bad = G.Problem(7, probs[0].profit, probs[0].weight, probs[0].capacity, probs[0].density)
    assert B.pbit_batch_workspace_bytes([probs[1], bad], pars[:2]) == 0
    st = lib.pbit_create_batch(None, None, 0, None, 0, None, 0, None, ctypes.byref(ctypes.c_void_p()))
    assert st == B.PBIT_EINVAL
    ms = B._MarshalledSet([probs[1], bad], pars[:2])
    h = ctypes.c_void_p()
    st = lib.pbit_create_batch(ms.problems, ms.params, 2, None, 0, None, 0, None, ctypes.byref(h))
    assert st == B.PBIT_EINVAL and b"member 1" in lib.pbit_last_error()


def test_philox_counter_bound_at_the_boundary(lib):
    """Sweeps x ceil(n_ext/4) beyond 2^32 would wrap the counter word
    t ceil(n_ext/4) + i/4 and replay draws: PBIT_ERANGE, exactly where the
    oracle refuses the same settings."""
    prob = G.mkp(1400, 32, G.rng_for(961, 2))
    par = G.Params(replicas=1, sweeps=1, beta=Fraction(50), alpha=Fraction(5))
    nq = (B.pbit_plan(prob, par).n_ext + 3) // 4
    T_ok = (1 << 32) // nq
    assert T_ok < (1 << 24)
    B.pbit_plan(prob, G.Params(replicas=1, sweeps=T_ok, beta=Fraction(50), alpha=Fraction(5)))
    _expect(B.PBIT_ERANGE, prob, G.Params(replicas=1, sweeps=T_ok + 1, beta=Fraction(50), alpha=Fraction(5)))
    with pytest.raises(O.OracleRangeError):
        O.build_program(prob, G.Params(replicas=1, sweeps=T_ok + 1, beta=Fraction(50), alpha=Fraction(5)))


def test_round_output_layout_has_the_saturation_word(lib):
    prob, par, _ = G.workload(0, 0)
    info = B.pbit_plan(prob, par)
    assert info.out_round < info.out_sat < info.out_bytes
    assert info.out_sat % 256 == 0


def test_diminishing_step_settings_are_validated(lib):
    """eta_decay_rounds outside [0, 2^20] is refused; inside it plans."""
    prob, par, _ = G.workload(0, 0)
    for bad in (-1, (1 << 20) + 1):
        _expect(B.PBIT_EINVAL, prob, G.Params(replicas=64, sweeps=10, eta_decay=bad))
    for ok in (0, 1, 1 << 20):
        B.pbit_plan(prob, G.Params(replicas=64, sweeps=10, eta_decay=ok))


def test_parallel_tempering_settings_and_plan(lib):
    """pt_slots: refused where the oracle refuses it; the multiplier range is
    the oracle's (narrowed for the exchange's energies); the round outputs
    carry the ladder positions."""
    prob = G.qkp(40, Fraction(1, 2), G.rng_for(962, 0))
    for bad in (dict(pt_slots=3), dict(pt_slots=4, replicas=66), dict(pt_slots=4, fixed_beta=True),
                dict(pt_slots=4, beta=Fraction(0))):
        kw = dict(replicas=64, sweeps=10, beta=Fraction(5))
        kw.update(bad)
        _expect(B.PBIT_EINVAL, prob, G.Params(**kw))
        with pytest.raises(ValueError):
            O.build_program(prob, G.Params(**kw))
    _expect(B.PBIT_EINVAL, G.mkp(30, 3, G.rng_for(962, 1)), G.Params(replicas=64, sweeps=10, pt_slots=4))
    for L in (2, 8, 64):
        par = G.Params(replicas=128, sweeps=10, beta=Fraction(7), pt_slots=L)
        info = B.pbit_plan(prob, par)
        prog = O.build_program(prob, par)
        assert info.lq_max == prog.lq_max and info.shift == prog.S
        assert info.out_slot < info.out_bytes
    # batches run annealing members only
    par = G.Params(replicas=64, sweeps=10, beta=Fraction(7), pt_slots=4)
    assert B.pbit_batch_workspace_bytes([prob, prob], [G.Params(replicas=64, sweeps=10), par]) == 0
    assert "single instances" in lib.pbit_last_error().decode()
