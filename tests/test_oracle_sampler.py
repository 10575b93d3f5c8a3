"""Pins of the oracle's sampler: local-field identity, threshold table, Philox,
exact law of the quantised chain, Boltzmann statistics and special cases."""
import math
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import brute as BF
from oracle import oracle as O
from paper_2501_04971_amd import generators as G

HERE = os.path.dirname(os.path.abspath(__file__))


def _prog(prob, **kw):
    par = G.Params(**kw)
    return O.build_program(prob, par)


# ---------------------------------------------------------------- field

@pytest.mark.parametrize("which", ["tiny-qkp", "tiny-mkp", "qkp-100", "mkp-250", "mkp-500-30"])
def test_local_field_is_energy_difference(which):
    """Z_i = -D (L(x, x_i=1) - L(x, x_i=0)) with L evaluated from its definition
    (Eq. Lagrange_energy with Eq. penalty_energy)."""
    rng = np.random.default_rng(11)
    if which == "tiny-qkp":
        prob = G.tiny(7, 1, True, G.rng_for(901, 0))
    elif which == "tiny-mkp":
        prob = G.tiny(6, 3, False, G.rng_for(901, 1))
    elif which == "qkp-100":
        prob = G.family0(0)
    elif which == "mkp-250":
        prob = G.family1(0)
    else:
        prob = G.mkp(500, 30, G.rng_for(901, 2))
    prog = _prog(prob)
    sites = range(prog.n_ext) if prog.n_ext < 40 else rng.choice(prog.n_ext, 12, replace=False)
    for trial in range(3):
        x = rng.integers(0, 2, size=prog.n_ext)
        lq = [int(v) for v in rng.integers(-prog.lq_max // 64, prog.lq_max // 64, size=prog.m)]
        for i in sites:
            x1 = x.copy(); x1[i] = 1
            x0 = x.copy(); x0[i] = 0
            expect = -(O.energy(prog, x1, lq) - O.energy(prog, x0, lq))
            assert O.local_field(prog, x, lq, int(i)) == expect
            assert abs(expect) < (1 << 62)


def test_index_grid_matches_beta_and_rounding():
    """idx = round(beta_t Z / (2 s_f s_g^2)) to within the grid error, computed
    identically by the C (int128 floor division) and Python (big-int shift) forms."""
    rng = np.random.default_rng(2)
    prog = _prog(G.family0(1), sweeps=50)
    betas = prog.beta_values()
    for _ in range(2000):
        t = int(rng.integers(0, prog.T))
        Z = int(rng.integers(-(1 << 50), 1 << 50)) >> int(rng.integers(0, 40))
        i_c = O.index_c(prog, Z, t)
        assert i_c == O.index_of(prog, Z, t)
        exact = Fraction(Z) * Fraction(prog.beta_values()[t]) / (2 * prog.s_f * prog.s_g ** 2)
        if abs(exact) < 2300:
            assert abs(i_c - exact) <= Fraction(1, 2)
    # grid value vs intended beta: relative error below 2^-29 at the end of the run
    beta_true = Fraction(5)
    assert abs(betas[-1] - beta_true) / beta_true < Fraction(1, 1 << 29)


# ---------------------------------------------------------------- table, rng

def test_theta_table_closed_form():
    """Theta[j] = round(2^24 (1 + tanh(j/256)) / 2): exact centre, symmetry,
    monotonicity, saturation, and agreement with float tanh."""
    th = O.theta_table()
    H = O.THETA_HALF
    assert len(th) == 2 * H + 1
    assert th[H] == 1 << 23
    assert th[0] == 0 and th[-1] == 1 << 24
    for j in range(H + 1):
        assert th[H + j] + th[H - j] == 1 << 24
    assert all(a <= b for a, b in zip(th, th[1:]))
    for j in range(-H, H + 1, 7):
        v = (1 << 24) * (1.0 + math.tanh(j / 256.0)) / 2.0
        assert abs(th[H + j] - v) <= 0.5 + 1e-6


def _rocrand_ref():
    exe = os.path.join(HERE, "_build", "philox_rocrand")
    src = os.path.join(HERE, "philox_rocrand.cpp")
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(src):
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        if not os.path.exists(hipcc):
            pytest.skip("hipcc not available for the rocRAND cross-check")
        os.makedirs(os.path.dirname(exe), exist_ok=True)
        subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", src, "-o", exe], check=True,
                       capture_output=True)
    return exe


def test_philox_matches_rocrand():
    """The oracle's Philox4x32-10 equals rocRAND's independent implementation."""
    exe = _rocrand_ref()
    rng = np.random.default_rng(7)
    rows = [[0] * 6, [0xFFFFFFFF] * 6] + rng.integers(0, 1 << 32, size=(200, 6)).tolist()
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [[int(v) for v in line.split()] for line in out.strip().splitlines()]
    for r, e in zip(rows, ref):
        assert O.philox(r[:4], r[4:]) == e


def test_counter_layout_replica_independence():
    """Counters are (sweep/site group, round, replica, instance): a replica's run
    does not depend on which other replicas run beside it."""
    prog = _prog(G.family0(2), sweeps=30, replicas=16)
    xa, ga = O.sa_round(prog, [0], 3, 0, 16, 4)
    xb, gb = O.sa_round(prog, [0], 3, 9, 1, 1)
    assert (xa[9] == xb[0]).all() and (ga[9] == gb[0]).all()
    xc, _ = O.sa_round(prog, [0], 4, 0, 16, 4)
    assert not (xa == xc).all()


# ---------------------------------------------------------------- statistics

def _chi2_pvalue(counts, probs, min_expected=5.0):
    counts = np.asarray(counts, dtype=float)
    exp = np.asarray(probs) * counts.sum()
    order = np.argsort(exp)
    c_acc = e_acc = 0.0
    obs, ex = [], []
    for j in order:
        c_acc += counts[j]
        e_acc += exp[j]
        if e_acc >= min_expected:
            obs.append(c_acc); ex.append(e_acc); c_acc = e_acc = 0.0
    if e_acc > 0:
        obs[-1] += c_acc; ex[-1] += e_acc
    chi2 = sum((o - e) ** 2 / e for o, e in zip(obs, ex))
    return float(stats.chi2.sf(chi2, len(obs) - 1))


def _state_codes(x):
    return (x.astype(np.int64) << np.arange(x.shape[1])).sum(axis=1)


@pytest.mark.parametrize("quad", [True, False])
def test_run_law_matches_exact_chain(quad):
    """Final states of many annealing runs follow the exact law of the
    quantised sequential Gibbs chain computed from the energy definition."""
    if quad:
        prob = G.tiny(4, 1, True, G.rng_for(902, 0), pmax=5, wmax=5)
    else:
        prob = G.tiny(4, 2, False, G.rng_for(902, 1), pmax=5, wmax=3)
    R = 60000
    prog = _prog(prob, replicas=R, sweeps=6, beta=Fraction(3), p_q=256 * 2)
    assert prog.n_ext <= 10
    lq = [256 + 37 * k for k in range(prog.m)]
    law = BF.exact_run_law(prog, lq)
    x, _ = O.sa_round(prog, lq, 0, 0, R, os.cpu_count())
    counts = np.bincount(_state_codes(x), minlength=len(law))
    assert _chi2_pvalue(counts, law) > 1e-4
    # a deliberately wrong law (the unquantised chain at twice the beta) is rejected
    prog2 = _prog(prob, replicas=R, sweeps=6, beta=Fraction(6), p_q=256 * 2)
    assert _chi2_pvalue(counts, BF.exact_run_law(prog2, lq)) < 1e-6


def test_beta_zero_gives_fair_coins():
    """At beta = 0 every spin is an independent fair coin (Theta[0] = 2^23)."""
    prob = G.tiny(5, 1, True, G.rng_for(903, 0))
    R = 40000
    prog = _prog(prob, replicas=R, sweeps=3, beta=Fraction(0), fixed_beta=True)
    x, _ = O.sa_round(prog, [0], 0, 0, R, os.cpu_count())
    counts = np.bincount(_state_codes(x), minlength=1 << prog.n_ext)
    uniform = np.full(1 << prog.n_ext, 1.0 / (1 << prog.n_ext))
    assert _chi2_pvalue(counts, uniform) > 1e-4


def test_stationary_law_is_boltzmann():
    """At fixed beta the quantised sweep operator's stationary law is close to
    exp(-beta L) / Z (Eq. Boltzmann_distrib); a factor-2 error in the p-bit
    input would give exp(-2 beta L) and fail."""
    prob = G.tiny(4, 1, True, G.rng_for(904, 0), pmax=4, wmax=4)
    beta = Fraction(2)
    prog = _prog(prob, replicas=1, sweeps=1, beta=beta, fixed_beta=True, p_q=256)
    lq = [128]
    pi = BF.stationary(BF.sweep_matrix(prog, lq, 0))
    tv = 0.5 * np.abs(pi - BF.boltzmann(prog, lq, beta)).sum()
    tv2 = 0.5 * np.abs(pi - BF.boltzmann(prog, lq, 2 * beta)).sum()
    assert tv < 0.01
    assert tv2 > 5 * tv


def test_single_spin_closed_form():
    """One spin (no slack): P(x = 1) = (1 + tanh(beta I)) / 2 with I = Z / (2D)."""
    prob = G.Problem(G.KIND_MKP, np.array([3], dtype=np.int32), np.array([[2]], dtype=np.int32),
                     np.array([0], dtype=np.int64))
    for beta in [Fraction(1, 2), Fraction(2), Fraction(7)]:
        prog = _prog(prob, replicas=1, sweeps=1, beta=beta, fixed_beta=True, p_q=256 * 3)
        assert prog.n_ext == 1
        lq = [-300]
        Z = O.local_field(prog, [0], lq, 0)
        p_table = O.theta_table()[O.index_of(prog, Z, 0) + O.THETA_HALF] / float(1 << 24)
        p_exact = 0.5 * (1.0 + math.tanh(float(beta) * Z / (2.0 * prog.D)))
        assert abs(p_table - p_exact) < 1.0 / 1000


def test_large_beta_is_coordinate_descent():
    """With a huge beta every visit is a greedy move: the final state admits no
    single flip that lowers L."""
    prob = G.family0(3)
    prog = _prog(prob, replicas=4, sweeps=40, beta=Fraction(10 ** 7), fixed_beta=True)
    lq = [prog.lq_max // 8]
    x, _ = O.sa_round(prog, lq, 0, 0, 4, 4)
    for r in range(4):
        e0 = O.energy(prog, x[r], lq)
        for i in range(0, prog.n_ext, 5):
            y = x[r].copy(); y[i] ^= 1
            assert O.energy(prog, y, lq) >= e0


# ---------------------------------------------------------------- lambda step

def test_lambda_step_tracks_algorithm_1():
    """With R = 1 the integer multiplier follows lambda <- lambda + eta g/s_g of
    Algorithm 1 to within the rounding of its 2^-32 accumulator, and it moves
    up while the knapsack is overfull."""
    prog = _prog(G.family1(0), replicas=1, eta=Fraction(1, 20))
    rng = np.random.default_rng(4)
    acc = [0] * prog.m
    exact = [Fraction(0)] * prog.m
    for step in range(1, 200):
        G_ = [int(v) for v in rng.integers(-5000, 40000, size=prog.m)]
        prev = list(acc)
        acc, lq = O.lambda_step(prog, acc, G_, 1)
        exact = [e + prog.eta * Fraction(gk, prog.s_g) for e, gk in zip(exact, G_)]
        for a, e, lqk in zip(acc, exact, lq):
            assert abs(Fraction(a, 1 << 32) - e) <= Fraction(step, 1 << 33)
            assert abs(Fraction(lqk, 256) - Fraction(a, 1 << 32)) <= Fraction(1, 512)
        for a, p, gk in zip(acc, prev, G_):
            assert (a > p) == (gk > 0) or gk == 0


def test_lambda_step_symmetry_and_clamp():
    prog = _prog(G.family0(0), replicas=64)
    a1, l1 = O.lambda_step(prog, [0], [12345], 64)
    a2, l2 = O.lambda_step(prog, [0], [-12345], 64)
    assert a1 == [-v for v in a2] and l1 == [-v for v in l2]
    cap = prog.lq_max << 24
    a3, l3 = O.lambda_step(prog, [cap - 5], [10 ** 9], 64)
    assert a3 == [cap] and l3 == [prog.lq_max]
