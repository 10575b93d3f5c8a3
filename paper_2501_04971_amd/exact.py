"""Exact optima of knapsack instances: the OPT of the accuracy metric.

The paper scores a feasible sample by its cost relative to the optimum
(Sec. IV-A, Eq. accuracy) and obtains MKP optima by branch and bound
(Sec. IV-B, Table 5).  This module does the same on the host: branch and bound
by the HiGHS mixed-integer solver (scipy.optimize.milp) at zero relative gap on

* MKP: the integer program itself, max c.x s.t. A x <= b, x in {0,1}^n;
* QKP: the standard linearisation, one variable y_ij in [0, 1] per pair with
  p_ij != 0 and profit sum_i p_ii x_i + sum_{i<j} p_ij y_ij, with
  y_ij <= x_i, y_ij <= x_j for p_ij > 0 (y_ij = x_i x_j at an optimum, since
  y is maximised) and y_ij >= x_i + x_j - 1 for p_ij < 0 (y minimised).

The solver's answer is not taken on trust: the returned assignment is
re-scored in exact integers (profit and every constraint), and the optimum is
reported as proven only when the solver's dual bound is below that profit + 1
(profits are integers).  The evaluation drivers use it; it is not on the
sampling path.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from .generators import KIND_MKP, KIND_QKP, Problem


@dataclass
class Optimum:
    profit: int | None     # None when no feasible assignment exists
    x: np.ndarray | None   # 0/1 bytes, length n
    proven: bool           # dual bound < profit + 1
    bound: float           # solver's dual bound on the profit
    seconds: float


def profit_of(prob: Problem, x: np.ndarray) -> int:
    """Objective of Sec. IV-A / IV-B in exact integers (each pair once)."""
    x = np.asarray(x, dtype=np.int64)
    if prob.kind == KIND_QKP:
        P = np.asarray(prob.profit, dtype=np.int64).reshape(prob.n, prob.n)
        return int(np.diag(P) @ x + (x @ np.triu(P, 1) @ x))
    return int(np.asarray(prob.profit, dtype=np.int64) @ x)


def feasible(prob: Problem, x: np.ndarray) -> bool:
    A = np.asarray(prob.weight, dtype=np.int64).reshape(prob.m, prob.n)
    return bool((A @ np.asarray(x, dtype=np.int64) <= np.asarray(prob.capacity, dtype=np.int64)).all())


def solve(prob: Problem, time_limit: float = 3600.0) -> Optimum:
    """Maximum profit over feasible assignments (branch and bound, zero gap)."""
    from scipy.optimize import Bounds, LinearConstraint, milp
    from scipy.sparse import coo_matrix

    n, m = prob.n, prob.m
    A = np.asarray(prob.weight, dtype=np.float64).reshape(m, n)
    b = np.asarray(prob.capacity, dtype=np.float64)
    rows, cols, vals, lo, hi = [], [], [], [], []

    def add_row(entries, lower, upper):
        r = len(lo)
        for c, v in entries:
            rows.append(r)
            cols.append(c)
            vals.append(v)
        lo.append(lower)
        hi.append(upper)

    for k in range(m):
        add_row([(i, A[k, i]) for i in range(n) if A[k, i] != 0], -np.inf, b[k])
    if prob.kind == KIND_QKP:
        P = np.asarray(prob.profit, dtype=np.int64).reshape(n, n)
        iu, ju = np.nonzero(np.triu(P, 1))
        nv = n + len(iu)
        c = np.zeros(nv)
        c[:n] = -np.diag(P)
        for e, (i, j) in enumerate(zip(iu, ju)):
            y = n + e
            c[y] = -P[i, j]
            if P[i, j] > 0:
                add_row([(y, 1.0), (int(i), -1.0)], -np.inf, 0.0)
                add_row([(y, 1.0), (int(j), -1.0)], -np.inf, 0.0)
            else:
                add_row([(y, 1.0), (int(i), -1.0), (int(j), -1.0)], -1.0, np.inf)
    elif prob.kind == KIND_MKP:
        nv = n
        c = -np.asarray(prob.profit, dtype=np.float64)
    else:
        raise ValueError("unknown problem kind")
    integrality = np.zeros(nv)
    integrality[:n] = 1
    cons = LinearConstraint(coo_matrix((vals, (rows, cols)), shape=(len(lo), nv)).tocsr(), lo, hi)
    t0 = time.perf_counter()
    res = milp(c, constraints=cons, integrality=integrality, bounds=Bounds(0, 1),
               options={"time_limit": time_limit, "mip_rel_gap": 0.0, "disp": False})
    dt = time.perf_counter() - t0
    bound = -float(getattr(res, "mip_dual_bound", np.nan)) if getattr(res, "mip_dual_bound", None) is not None \
        else np.inf
    if res.x is None:
        # infeasible only if the empty selection is infeasible (capacities < 0)
        return Optimum(None, None, res.status == 2, bound, dt)
    x = (np.asarray(res.x[:n]) > 0.5).astype(np.uint8)
    if not feasible(prob, x):
        raise RuntimeError("solver returned an infeasible assignment")
    p = profit_of(prob, x)
    proven = res.status == 0 and bound < p + 1
    return Optimum(p, x, bool(proven), bound, dt)
