"""The per-element rounding bounds of the set encoder's GPU test (net_bounds)
checked on the CPU: they accept the oracle's own rounding (every stored value
rounded once from an exact sum, which the device's fp32 sums must bracket),
and they reject a planted one-ulp error in a stored activation and a planted
error of three bounds in one gradient entry."""
import numpy as np
import pytest

from oracle import lambda_net as N
from paper_2501_04971_amd import binding as B

import net_bounds as NB
from test_net_gpu import bf_bits_to_f64, oracle_sets, problems


def oracle_as_device(pk, w, y32):
    wq = N.bf16(w)
    sets = oracle_sets(pk)
    t, (Wq, cache) = N.forward(w, sets, quant=True)
    loss, _, grad = N.backward(w, sets, y32.astype(np.float64), quant=True)
    x = bf_bits_to_f64(pk["x"])
    ctx = bf_bits_to_f64(pk["ctx"])
    rows = pk["rows"]
    H1 = np.zeros((rows, N.HID))
    H2 = np.zeros((rows, N.HID))
    Z = np.zeros((pk["sets"], N.Z_IN))
    G1 = np.zeros((pk["sets"], N.HID))
    dP = np.zeros((pk["sets"], N.HID))
    r = t - y32.astype(np.float64)
    dt = N.huber_grad(r) / pk["sets"]
    for s, (Xq, h1, h2, z, g1) in enumerate(cache):
        r0, n = pk["set_rows"][s], pk["set_n"][s]
        H1[r0:r0 + n], H2[r0:r0 + n], Z[s], G1[s] = h1, h2, z, g1
        Z[s, N.HID:] = ctx[s]
        dP[s] = Wq["W3"][:, :N.HID].T @ (dt[s] * Wq["w4"] * (g1 > 0))
    dev = {"X": x, "ctx": ctx, "H1": H1, "H2": H2, "Z": Z, "G1": G1, "t": t, "loss": loss, "dP": dP,
           "grad": grad}
    return wq, dev


@pytest.fixture(scope="module")
def case():
    ms = problems()[:4]
    pk = B.pbit_net_pack([p for p, _ in ms], [q for _, q in ms])
    w = N.init_params(3)
    y32 = (np.random.default_rng(3).normal(size=pk["sets"]) * 1.5).astype(np.float32)
    return pk, w, y32


def test_bounds_accept_the_oracles_rounding(case):
    pk, w, y32 = case
    wq, dev = oracle_as_device(pk, w, y32)
    worst = NB.check(pk, wq, y32, dev)
    assert worst < 1e-3  # far tighter than a percent of each group's largest entry


def test_bounds_reject_a_one_ulp_activation_error(case):
    pk, w, y32 = case
    wq, dev = oracle_as_device(pk, w, y32)
    h = dev["H2"]
    i = tuple(np.argwhere(h > 0)[7])
    h[i] += 2.0 ** (np.floor(np.log2(h[i])) - 7)  # the next bf16 value up (7 fraction bits)
    assert N.bf16(h[i]) == h[i]
    with pytest.raises(AssertionError, match="H2"):
        NB.check(pk, wq, y32, dev)


def test_bounds_reject_a_small_gradient_error(case):
    pk, w, y32 = case
    wq, dev = oracle_as_device(pk, w, y32)
    g = N.unflatten(dev["grad"])
    # a small entry of dW1, well inside a percent of the group's largest one
    k = np.argsort(np.abs(g["W1"]).ravel())[len(g["W1"].ravel()) // 2]
    scale = np.abs(g["W1"]).max()
    g["W1"].ravel()[k] += 1e-4 * scale
    dev["grad"] = N.flatten(g)
    with pytest.raises(AssertionError, match="gradient W1"):
        NB.check(pk, wq, y32, dev)
