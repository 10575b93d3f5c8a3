"""Per-element rounding bounds for the set encoder's kernels (test helper).

The kernels store bf16 activations and accumulate in fp32; the oracle's
precision model says where they round.  Given the device's own stored
activations (the workspace layout of pbit_net_workspace_bytes), every
quantity of the next layer is bounded element by element:

* an fp32 accumulation of k terms of exactly representable products
  (bf16 x bf16, or bf16 x fp32 where stated) differs from the exact sum by at
  most gamma_k * sum |terms|, gamma_k = k u / (1 - k u), u = 2^-24, in any
  order (Higham, Accuracy and Stability of Numerical Algorithms, 2nd ed.,
  Sec. 4.2; a fused multiply-add only removes roundings);
* a stored bf16 value is the round-to-nearest-even image of its fp32 value,
  so it lies between the images of the two ends of that value's interval
  (rounding is monotone);
* where a rounded intermediate is not stored (the backward pass's dH2 and
  dH1), the set of its possible bf16 values is carried on as an interval
  (midpoint, radius) into the sums that use it.

check() raises AssertionError naming the first element outside its bound.
Only numpy; nothing from the library."""
from __future__ import annotations

import numpy as np

from oracle import lambda_net as N

U = 2.0 ** -24


def gamma(k: int) -> float:
    return k * U / (1.0 - k * U)


def bf(v):
    return N.bf16(v)


def _interval_of_rounding(lo, hi):
    """Midpoint and radius of [bf16(lo), bf16(hi)]."""
    a, b = bf(lo), bf(hi)
    return (a + b) / 2.0, (b - a) / 2.0


def _in_rounding(dev, lo, hi, what):
    a, b = bf(lo), bf(hi)
    bad = (dev < a) | (dev > b)
    if bad.any():
        i = tuple(np.argwhere(bad)[0])
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} outside their rounding interval; "
                             f"first {i}: {dev[i]!r} not in [{a[i]!r}, {b[i]!r}]")


def _close(dev, m, r, what):
    r = r + U * np.abs(m) + 1e-30  # the final fp32 rounding
    bad = np.abs(dev - m) > r
    if bad.any():
        i = tuple(np.argwhere(bad)[0])
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} outside their bound; "
                             f"first {i}: {dev[i]!r} vs {m[i]!r} +- {r[i]!r}")


def relu(v):
    return np.maximum(v, 0.0)


def check(pk, wq, y32, dev):
    """pk: pbit_net_pack output; wq: the bf16 weights as float64 (flat);
    y32: float32 targets; dev: dict of the device's float64 values
      X (rows, 16), ctx (sets, 16), H1, H2 (rows, 128), Z (sets, 144),
      G1 (sets, 128), t (sets,), loss (scalar), dP (sets, 128), grad (flat).
    Returns the largest bound relative to its group's max |value| (how tight)."""
    p = N.unflatten(wq)
    W1, b1, W2, b2 = p["W1"], p["b1"], p["W2"], p["b2"]
    W3, b3, w4, b4 = p["W3"], p["b3"], p["w4"], float(p["b4"][0])
    S = pk["sets"]
    X, H1, H2, Z, G1 = dev["X"], dev["H1"], dev["H2"], dev["Z"], dev["G1"]
    t = dev["t"]
    # ---- forward, layer by layer from the device's own inputs
    for s in range(S):
        r0, n = int(pk["set_rows"][s]), int(pk["set_n"][s])
        Xs, H1s, H2s = X[r0:r0 + n], H1[r0:r0 + n], H2[r0:r0 + n]
        m = Xs @ W1.T + b1
        r = gamma(N.F_IN + 1) * (np.abs(Xs) @ np.abs(W1).T + np.abs(b1))
        _in_rounding(H1s, relu(m - r), relu(m + r), f"H1 of set {s}")
        m = H1s @ W2.T + b2
        r = gamma(N.HID + 1) * (np.abs(H1s) @ np.abs(W2).T + np.abs(b2))
        _in_rounding(H2s, relu(m - r), relu(m + r), f"H2 of set {s}")
        # mean: an fp32 sum of n bf16 values, then one division
        m = H2s.sum(axis=0) / n
        r = gamma(n) * np.abs(H2s).sum(axis=0) / n + 2 * U * np.abs(m)
        _in_rounding(Z[s, :N.HID], m - r, m + r, f"pooled mean of set {s}")
        assert (Z[s, N.HID:] == dev["ctx"][s]).all(), f"context of set {s}"
        m = W3 @ Z[s] + b3
        r = gamma(N.Z_IN + 1) * (np.abs(W3) @ np.abs(Z[s]) + abs(b3))
        _in_rounding(G1[s], relu(m - r), relu(m + r), f"G1 of set {s}")
    m = G1 @ w4 + b4
    r = gamma(N.HID + 1) * (np.abs(G1) @ np.abs(w4) + abs(b4))
    _close(t, m, r, "t")
    # ---- loss and dt from the device's t (fp32: t - y, clip, / S)
    res = t - y32.astype(np.float64)
    hub = N.huber(res)
    # fp32: t - y, the Huber term, a sum of S, one division
    _close(np.array([dev["loss"]]), np.array([hub.mean()]), np.array([gamma(S + 8) * hub.mean()]), "loss")
    dt_m = np.clip(res, -N.HUBER_DELTA, N.HUBER_DELTA) / S
    dt_r = 3 * U * np.abs(dt_m)
    # ---- head gradients (products with an fp32 factor are rounded once more)
    g = {}
    mask1 = (G1 > 0).astype(np.float64)
    g["w4"] = (dt_m @ G1, dt_r @ np.abs(G1) + gamma(S + 1) * (np.abs(dt_m) + dt_r) @ np.abs(G1))
    g["b4"] = (np.array([dt_m.sum()]), np.array([dt_r.sum() + gamma(S) * (np.abs(dt_m) + dt_r).sum()]))
    dG1_m = dt_m[:, None] * w4[None, :] * mask1
    dG1_r = dt_r[:, None] * np.abs(w4)[None, :] * mask1 + U * np.abs(dG1_m)
    g["W3"] = (dG1_m.T @ Z, dG1_r.T @ np.abs(Z) + gamma(S + 1) * (np.abs(dG1_m) + dG1_r).T @ np.abs(Z))
    g["b3"] = (dG1_m.sum(axis=0), dG1_r.sum(axis=0) + gamma(S) * (np.abs(dG1_m) + dG1_r).sum(axis=0))
    Wp = W3[:, :N.HID]
    m = dG1_m @ Wp
    r = dG1_r @ np.abs(Wp) + gamma(N.HID + 1) * (np.abs(dG1_m) + dG1_r) @ np.abs(Wp)
    _close(dev["dP"], m, r, "dP")
    # ---- phi gradients from the device's dP: dH2 = bf16(dP / n) on active units,
    # dH1 = bf16((dH2 W2) on active units), both carried as intervals
    acc = {k: [0.0, 0.0] for k in ("W2", "b2", "W1", "b1")}
    rows_total = 0
    for s in range(S):
        r0, n = int(pk["set_rows"][s]), int(pk["set_n"][s])
        Xs, H1s, H2s = X[r0:r0 + n], H1[r0:r0 + n], H2[r0:r0 + n]
        rows_total += n
        q = dev["dP"][s] / n
        h2m, h2r = _interval_of_rounding(q - 2 * U * np.abs(q), q + 2 * U * np.abs(q))
        a2 = (H2s > 0).astype(np.float64)
        dH2m, dH2r = a2 * h2m[None, :], a2 * h2r[None, :]
        acc["W2"][0] = acc["W2"][0] + dH2m.T @ H1s
        acc["W2"][1] = acc["W2"][1] + dH2r.T @ np.abs(H1s)
        acc["b2"][0] = acc["b2"][0] + dH2m.sum(axis=0)
        acc["b2"][1] = acc["b2"][1] + dH2r.sum(axis=0)
        pm = dH2m @ W2
        pr = dH2r @ np.abs(W2) + gamma(N.HID) * (np.abs(dH2m) + dH2r) @ np.abs(W2)
        a1 = (H1s > 0).astype(np.float64)
        h1m, h1r = _interval_of_rounding(pm - pr, pm + pr)
        dH1m, dH1r = a1 * h1m, a1 * h1r
        acc["W1"][0] = acc["W1"][0] + dH1m.T @ Xs
        acc["W1"][1] = acc["W1"][1] + dH1r.T @ np.abs(Xs)
        acc["b1"][0] = acc["b1"][0] + dH1m.sum(axis=0)
        acc["b1"][1] = acc["b1"][1] + dH1r.sum(axis=0)
        # accumulation error of the sums over rows, added below from |terms|
        acc.setdefault("absW2", 0.0)
        acc["absW2"] = acc["absW2"] + (np.abs(dH2m) + dH2r).T @ np.abs(H1s)
        acc.setdefault("absb2", 0.0)
        acc["absb2"] = acc["absb2"] + (np.abs(dH2m) + dH2r).sum(axis=0)
        acc.setdefault("absW1", 0.0)
        acc["absW1"] = acc["absW1"] + (np.abs(dH1m) + dH1r).T @ np.abs(Xs)
        acc.setdefault("absb1", 0.0)
        acc["absb1"] = acc["absb1"] + (np.abs(dH1m) + dH1r).sum(axis=0)
    ga = gamma(rows_total)
    for k in ("W2", "b2", "W1", "b1"):
        g[k] = (acc[k][0], acc[k][1] + ga * acc["abs" + k])
    gd = N.unflatten(dev["grad"])
    worst = 0.0
    for name, _ in N.LAYOUT:
        m, r = g[name]
        m = np.broadcast_to(m, gd[name].shape)
        r = np.broadcast_to(r, gd[name].shape)
        _close(gd[name], m, r, f"gradient {name}")
        worst = max(worst, float(r.max() / max(np.abs(m).max(), 1e-30)))
    return worst
