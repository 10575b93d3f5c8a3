"""CPU ORACLE FOR THE LEARNED STARTING MULTIPLIERS -- TEST INFRASTRUCTURE ONLY.

Plain float64 numpy reference of the set encoder that predicts lambda_0 from an
instance, used by tests/ to check the library's HIP forward, backward and Adam
kernels and its host feature extraction.  Nothing in the product path imports
it, and it shares no code with the library.

The paper starts Algorithm 1 from lambda_0 = 0 and shows (Fig. 3, Sec. IV-A,
Sec. IV-B) that the multipliers settle to an instance-dependent lambda*.  The
network below is not in the paper: it maps an instance to a guess of lambda*
so that the loop can start near it.

Set encoder, one set per (instance, constraint k), one element per original
variable i:
  features (F = 16, five used, the rest zero):
    f0 = rho_i / (s_f n)         rho_i = h_i + sum_j W_ij  (profit row sum)
    f1 = n a_ki / b_k
    f2 = n mean_k' a_k'i / b_k'
    f3 = h_i / s_f
    f4 = clamp(ln(e_ki / rho_bar_k), -8, 8), e_ki = (h_i + sum_j W_ij / 2) / a_ki
         the item's profit per unit of weight k (+8 for a_ki = 0, -8 for e <= 0)
  context (C = 9): log(N_ext)/8, d, P_n/N_ext, beta_max/50, M/32, kind, and
    of the greedy fill of constraint k alone (items by decreasing e_ki, ties
    by index, until the first that does not fit): e of that item / rho_bar_k
    (0 if every item fits), b_k / sum_i a_ki, the items taken before it / n
  phi:  H1 = relu(X W1^T + b1), H2 = relu(H1 W2^T + b2)       (128 wide)
  pool: P = mean over the set's rows of H2
  head: z = [P, ctx, 0 pad] (144), G1 = relu(W3 z + b3), t = w4 . G1 + b4
  output: lambda_q,k = round_half_away(t * scale_k),
          scale_k = 256 rho_bar_k s_g / s_f,
          rho_bar_k = sum_i (h_i + sum_j W_ij / 2) / sum_i a_ki
  so t is a dimensionless multiplier: lambda in profit units per unit of
  constraint weight, relative to the mean profit per unit weight.

Precision model (the kernels' own): weights, inputs and every stored activation
(H1, H2, P, the context, G1) are bfloat16, products are accumulated exactly
here (float64) and in float32 on the device; t stays float32.  In the backward
pass dH2 = (dP / n_s) masked and dH1 = (dH2 W2) masked are rounded to
bfloat16 (they feed matrix-core products); everything else is float32.
quant=False switches every rounding off, which is what the finite-difference
checks use.

Loss: mean over sets of Huber(t - y) with delta = 1.
Adam (Kingma & Ba, 2015) on float32 master weights: beta1 0.9, beta2 0.999,
eps 1e-8, bias-corrected.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from paper_2501_04971_amd.generators import KIND_QKP

F_IN = 16
N_CTX = 9
Z_IN = 144
HID = 128
HUBER_DELTA = 1.0

# flat parameter layout: name, shape
LAYOUT = [("W1", (HID, F_IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, Z_IN)), ("b3", (HID,)), ("w4", (HID,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in LAYOUT)


def unflatten(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in LAYOUT:
        k = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def flatten(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in LAYOUT])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via float32, as the device
    rounds its float32 values; returns float64 holding the rounded values."""
    f = np.atleast_1d(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out.reshape(np.shape(x))


def _q(x, quant: bool):
    return bf16(x) if quant else np.asarray(x, dtype=np.float64)


# ---------------------------------------------------------------------------
# Features

@dataclass
class SetFeatures:
    X: np.ndarray       # (n, F_IN) float64, before rounding
    ctx: np.ndarray     # (N_CTX,)
    scale: float        # lambda_q = t * scale
    member: int
    k: int


def instance_features(prob, par, n_ext: int, pq: int, member: int = 0):
    """One SetFeatures per constraint of the instance (float64 values)."""
    n, m = prob.n, prob.m
    if prob.kind == KIND_QKP:
        Pm = np.asarray(prob.profit, dtype=np.float64).reshape(n, n)
        h = np.diag(Pm).copy()
        W = Pm - np.diag(h)
        d = float(prob.density)
    else:
        h = np.asarray(prob.profit, dtype=np.float64).reshape(n)
        W = np.zeros((n, n))
        d = 2.0 / (n_ext + 1)
    s_f = max(1.0, float(np.abs(np.asarray(prob.profit)).max()))
    A = np.asarray(prob.weight, dtype=np.float64).reshape(m, n)
    b = np.asarray(prob.capacity, dtype=np.float64).reshape(m)
    s_g = max(1.0, float(A.max(initial=0)), float(b.max(initial=0)))
    rho = h + W.sum(axis=1)
    ratio = A / np.maximum(b, 1.0)[:, None]
    mean_ratio = ratio.mean(axis=0)
    half = (h + 0.5 * W.sum(axis=1)).sum()
    ctx = np.array([math.log(n_ext) / 8.0, d, (pq / 256.0) / n_ext, float(par.beta) / 50.0,
                    m / 32.0, 0.0 if prob.kind == KIND_QKP else 1.0])
    hm = h + 0.5 * W.sum(axis=1)  # half-marginal profit of each item
    out = []
    for k in range(m):
        X = np.zeros((n, F_IN))
        X[:, 0] = rho / (s_f * n)
        X[:, 1] = n * ratio[k]
        X[:, 2] = n * mean_ratio
        X[:, 3] = h / s_f
        asum = A[k].sum()
        rho_bar = half / (asum if asum > 0 else 1.0)
        e = [math.inf if A[k, i] == 0 else float(hm[i]) / float(A[k, i]) for i in range(n)]
        for i in range(n):
            if e[i] == math.inf:
                X[i, 4] = 8.0
            elif e[i] <= 0.0 or rho_bar <= 0.0:
                X[i, 4] = -8.0
            else:
                X[i, 4] = min(8.0, max(-8.0, math.log(e[i] / rho_bar)))
        # greedy fill of constraint k alone
        order = sorted(range(n), key=lambda i: (-e[i], i))
        used, taken, e_break = 0.0, 0, 0.0
        for i in order:
            if used + A[k, i] > b[k]:
                e_break = e[i]
                break
            used += A[k, i]
            taken += 1
        greedy = [e_break / rho_bar if rho_bar > 0 else 0.0, b[k] / (asum if asum > 0 else 1.0), taken / n]
        out.append(SetFeatures(X, np.concatenate([ctx, greedy]), 256.0 * rho_bar * s_g / s_f, member, k))
    return out


# ---------------------------------------------------------------------------
# Network

def forward(flat, sets, quant: bool = True):
    """Returns (t per set, cache) for a list of (X, ctx) pairs."""
    p = unflatten(flat)
    Wq = {k: _q(v, quant) for k, v in p.items()}
    ts, cache = [], []
    for X, ctx in sets:
        Xq = _q(X, quant)
        H1 = _q(np.maximum(Xq @ Wq["W1"].T + Wq["b1"], 0.0), quant)
        H2 = _q(np.maximum(H1 @ Wq["W2"].T + Wq["b2"], 0.0), quant)
        P = _q(H2.mean(axis=0), quant)
        z = np.zeros(Z_IN)
        z[:HID] = P
        z[HID:HID + N_CTX] = _q(ctx, quant)
        G1 = _q(np.maximum(Wq["W3"] @ z + Wq["b3"], 0.0), quant)
        t = float(Wq["w4"] @ G1 + Wq["b4"][0])
        ts.append(t)
        cache.append((Xq, H1, H2, z, G1))
    return np.array(ts), (Wq, cache)


def huber(r):
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r)
    return np.where(a <= HUBER_DELTA, 0.5 * r * r, HUBER_DELTA * (a - 0.5 * HUBER_DELTA))


def huber_grad(r):
    return np.clip(np.asarray(r, dtype=np.float64), -HUBER_DELTA, HUBER_DELTA)


def loss(flat, sets, y, quant: bool = True) -> float:
    t, _ = forward(flat, sets, quant)
    return float(huber(t - np.asarray(y)).mean())


def backward(flat, sets, y, quant: bool = True):
    """(loss, t, flat gradient of the mean Huber loss)."""
    t, (Wq, cache) = forward(flat, sets, quant)
    S = len(sets)
    r = t - np.asarray(y, dtype=np.float64)
    dt = huber_grad(r) / S
    g = {name: np.zeros(shape) for name, shape in LAYOUT}
    for s, (Xq, H1, H2, z, G1) in enumerate(cache):
        g["w4"] += dt[s] * G1
        g["b4"][0] += dt[s]
        dG1 = dt[s] * Wq["w4"] * (G1 > 0)
        g["W3"] += np.outer(dG1, z)
        g["b3"] += dG1
        dP = Wq["W3"][:, :HID].T @ dG1
        n_s = H2.shape[0]
        dH2 = _q(dP / n_s, quant)[None, :] * (H2 > 0)
        g["W2"] += dH2.T @ H1
        g["b2"] += dH2.sum(axis=0)
        dH1 = _q((dH2 @ Wq["W2"]) * (H1 > 0), quant)
        g["W1"] += dH1.T @ Xq
        g["b1"] += dH1.sum(axis=0)
    return float(huber(r).mean()), t, flatten(g)


@dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    step: int = 0


def adam_init(n: int = N_PARAMS) -> AdamState:
    return AdamState(np.zeros(n), np.zeros(n), 0)


def adam_step(w, grad, st: AdamState, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update; returns the new weights (float64)."""
    st.step += 1
    st.m = beta1 * st.m + (1 - beta1) * grad
    st.v = beta2 * st.v + (1 - beta2) * grad * grad
    mh = st.m / (1 - beta1 ** st.step)
    vh = st.v / (1 - beta2 ** st.step)
    return np.asarray(w, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases (float32 values)."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shape in LAYOUT:
        if len(shape) == 2:
            lim = math.sqrt(6.0 / shape[1])
            parts[name] = rng.uniform(-lim, lim, size=shape)
        elif name == "w4":
            lim = math.sqrt(6.0 / HID)
            parts[name] = rng.uniform(-lim, lim, size=shape)
        else:
            parts[name] = np.zeros(shape)
    return flatten(parts).astype(np.float32).astype(np.float64)


def to_lambda_q(t: float, scale: float) -> int:
    """round_half_away(t * scale) computed in float64."""
    v = float(np.float32(t)) * scale
    return int(math.floor(abs(v) + 0.5)) * (1 if v >= 0 else -1)
