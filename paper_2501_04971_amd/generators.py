"""Seeded synthetic instance generators for QKP and MKP.

These are the only code shared by the product path and the CPU oracle: they draw
random integer problem data and hold none of the method's arithmetic (no
encoding, scaling, sampling or multiplier update).

The families follow the shapes the paper benchmarks on (Sec. IV-A: QKP with
N in {100,200,300} and W-density d in {0.25,0.5,0.75,1}; Sec. IV-B: MKP with
N in {100,250} and M in {5,10}).  The paper's own instance files are not
available, so these draws stand in for them:

* QKP: every pair i <= j (diagonal included) carries a profit p_ij ~ U{1..100}
  with probability d, mirrored to keep the matrix symmetric; item weights
  w_i ~ U{1..50}; capacity b ~ U{50..sum(w)}.
* MKP: weights a_ki ~ U{1..1000}; capacities b_k = floor(sum_i a_ki / 4);
  profits c_i = floor(sum_k a_ki / M + 500 u_i), u_i ~ U(0,1).

Every instance is drawn from numpy's PCG64 seeded by SeedSequence([family,
index]) so any (family, index) pair can be regenerated alone.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

KIND_QKP = 0
KIND_MKP = 1


@dataclass
class Problem:
    """Maximise profit(x) subject to weight @ x <= capacity, x in {0,1}^n.

    kind     KIND_QKP (profit is an n*n symmetric matrix whose diagonal holds the
             item values) or KIND_MKP (profit is a length-n vector).
    weight   (m, n) non-negative integers.
    capacity (m,) non-negative integers.
    density  nominal density of the pair-profit matrix (QKP); used by the
             penalty rule P = alpha*d*N.  Ignored for MKP.
    """

    kind: int
    profit: np.ndarray
    weight: np.ndarray
    capacity: np.ndarray
    density: Fraction = field(default_factory=lambda: Fraction(1))
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.weight.shape[1])

    @property
    def m(self) -> int:
        return int(self.weight.shape[0])


@dataclass
class Params:
    """Sampler settings for one instance (all in the paper's normalised units).

    replicas     independent chains sampled per round (they share lambda)
    sweeps       Monte-Carlo sweeps per annealing run (MCS per run)
    beta         beta_max of the linear 0 -> beta_max schedule
    eta          Lagrange step size
    p_q          256*P given directly, or None for the rule P = alpha*d*N
    alpha        the rule's constant (Table 1: 2 for QKP, 5 for MKP)
    seed         Philox key
    instance_id  last Philox counter word (tells instances of a batch apart)
    fixed_beta   hold beta at beta_max for every sweep (test mode)
    eta_decay    H: diminishing step eta H / (H + k) after round k; 0 = constant
    pt_slots     L > 0: parallel tempering instead of annealing, chains of L
                 replicas at the fixed ladder beta_max (j + 1) / L, j < L
    """

    replicas: int = 64
    sweeps: int = 1000
    beta: Fraction = Fraction(5)
    eta: Fraction = Fraction(1, 20)
    p_q: int | None = None
    alpha: Fraction = Fraction(2)
    seed: int = 0
    instance_id: int = 0
    fixed_beta: bool = False
    eta_decay: int = 0
    pt_slots: int = 0


def rng_for(family: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(family), int(index)])))


def qkp(n: int, density: Fraction | float, rng: np.random.Generator, name: str = "") -> Problem:
    d = Fraction(density).limit_denominator(1000)
    present = rng.random((n, n)) < float(d)
    values = rng.integers(1, 101, size=(n, n), dtype=np.int64)
    upper = np.triu(np.where(present, values, 0))
    p = upper + np.triu(upper, 1).T
    w = rng.integers(1, 51, size=n, dtype=np.int64)
    total = int(w.sum())
    b = int(rng.integers(min(50, total), total + 1))
    return Problem(KIND_QKP, p.astype(np.int32), w.reshape(1, n).astype(np.int32),
                   np.array([b], dtype=np.int64), d, name)


def mkp(n: int, m: int, rng: np.random.Generator, name: str = "") -> Problem:
    a = rng.integers(1, 1001, size=(m, n), dtype=np.int64)
    b = a.sum(axis=1) // 4
    u = rng.random(n)
    c = np.floor(a.sum(axis=0) / m + 500.0 * u).astype(np.int64)
    return Problem(KIND_MKP, c.astype(np.int32), a.astype(np.int32), b.astype(np.int64),
                   Fraction(1), name)


def tiny(n: int, m: int, quadratic: bool, rng: np.random.Generator, pmax: int = 9,
         wmax: int = 9) -> Problem:
    """Small random instance for enumeration tests (n + slack bits <= ~20)."""
    if quadratic:
        vals = rng.integers(0, pmax + 1, size=(n, n), dtype=np.int64)
        upper = np.triu(vals)
        p = upper + np.triu(upper, 1).T
        if p.max() == 0:
            p[0, 0] = 1
        profit = p.astype(np.int32)
        kind = KIND_QKP
    else:
        profit = rng.integers(1, pmax + 1, size=n, dtype=np.int64).astype(np.int32)
        kind = KIND_MKP
    a = rng.integers(1, wmax + 1, size=(m, n), dtype=np.int64)
    b = np.maximum(1, a.sum(axis=1) // 2)
    return Problem(kind, profit, a.astype(np.int32), b.astype(np.int64), Fraction(1, 2), "tiny")


# ---------------------------------------------------------------------------
# Workload families.  Family ids seed the generators.

def family0(index: int) -> Problem:
    """QKP, N=100, pair density 25%."""
    return qkp(100, Fraction(1, 4), rng_for(0, index), f"qkp-100-25-{index}")


def family1(index: int) -> Problem:
    """MKP, N=250, M=10."""
    return mkp(250, 10, rng_for(1, index), f"mkp-250-10-{index}")


def family2(index: int) -> Problem:
    """QKP, N=300, pair density 100%."""
    return qkp(300, Fraction(1), rng_for(2, index), f"qkp-300-100-{index}")


def family3(index: int) -> Problem:
    """Mixed batch member: even index -> QKP with N~U{100..300}, d in {.25,.5,.75,1};
    odd index -> MKP with N in {100,250,500}, M in {5,10,30}."""
    rng = rng_for(3, index)
    if index % 2 == 0:
        n = int(rng.integers(100, 301))
        d = [Fraction(1, 4), Fraction(1, 2), Fraction(3, 4), Fraction(1)][int(rng.integers(0, 4))]
        return qkp(n, d, rng, f"qkp-{n}-{int(d * 100)}-b{index}")
    n = [100, 250, 500][int(rng.integers(0, 3))]
    m = [5, 10, 30][int(rng.integers(0, 3))]
    return mkp(n, m, rng, f"mkp-{n}-{m}-b{index}")


FAMILIES = {0: family0, 1: family1, 2: family2, 3: family3}


# ---------------------------------------------------------------------------
# Workloads: (instance family, sampler settings, rounds).  Where a setting is
# not fixed by the workload description the paper's Table 1 value for that
# problem kind is used.

def workload(cfg: int, index: int = 0):
    """Returns (problem, params, rounds) for workload cfg and instance index."""
    if cfg == 0:
        return family0(index), Params(64, 1000, Fraction(5), Fraction(1, 20), None, Fraction(2)), 50
    if cfg == 1:
        return family1(index), Params(1024, 2000, Fraction(50), Fraction(1, 20), None, Fraction(5)), 100
    if cfg == 2:
        return family2(index), Params(4096, 5000, Fraction(5), Fraction(1, 20), None, Fraction(2)), 100
    if cfg == 3:
        prob = family3(index)
        if prob.kind == KIND_QKP:
            par = Params(256, 1000, Fraction(5), Fraction(1, 20), None, Fraction(2), instance_id=index)
            return prob, par, 50
        par = Params(256, 2000, Fraction(50), Fraction(1, 20), None, Fraction(5), instance_id=index)
        return prob, par, 100
    raise ValueError(f"unknown workload {cfg}")
