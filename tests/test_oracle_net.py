"""Pins of the learned-lambda_0 oracle against facts that do not come from the
oracle itself: central finite differences of its own loss (so a dropped term,
a wrong transpose or a wrong mask in the backward pass fails), set-encoder
invariances, closed forms of the Huber loss, of Adam's first steps and of the
bfloat16 rounding, and hand-computed features of a tiny instance."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import lambda_net as N
from oracle import oracle as O
from paper_2501_04971_amd import generators as G


def _sets(rng, sizes):
    out = []
    for n in sizes:
        X = np.zeros((n, N.F_IN))
        X[:, :4] = rng.normal(size=(n, 4))
        out.append((X, rng.normal(size=N.N_CTX)))
    return out


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    w = N.init_params(3) * 0.7
    sets = _sets(rng, [5, 9, 3])
    y = rng.normal(size=3) * 2
    _, _, grad = N.backward(w, sets, y, quant=False)
    # every parameter group, several coordinates each (biases of the hidden
    # layers included, which is where a dropped mask shows)
    o = 0
    picks = []
    for name, shape in N.LAYOUT:
        k = int(np.prod(shape))
        picks += [o + int(i) for i in rng.choice(k, size=min(k, 6), replace=False)]
        o += k
    h = 1e-6
    for i in picks:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (N.loss(wp, sets, y, quant=False) - N.loss(wm, sets, y, quant=False)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, grad[i])


def test_pooling_is_a_mean_over_the_set():
    rng = np.random.default_rng(2)
    w = N.init_params(5)
    X, ctx = _sets(rng, [7])[0]
    perm = rng.permutation(7)
    t1, _ = N.forward(w, [(X, ctx)], quant=False)
    t2, _ = N.forward(w, [(X[perm], ctx)], quant=False)
    assert abs(t1[0] - t2[0]) < 1e-12
    # a set of identical rows pools to that row
    t3, _ = N.forward(w, [(np.repeat(X[:1], 5, axis=0), ctx)], quant=False)
    t4, _ = N.forward(w, [(X[:1], ctx)], quant=False)
    assert abs(t3[0] - t4[0]) < 1e-12


def test_dead_relu_blocks_gradient():
    """With W1 negative and inputs positive every H1 is zero: no gradient
    reaches W1, b1 or W2 (the masks of both phi layers are exercised)."""
    rng = np.random.default_rng(3)
    p = N.unflatten(N.init_params(7))
    p["W1"] = -np.abs(p["W1"])
    p["b1"][:] = 0
    w = N.flatten(p)
    X = np.zeros((4, N.F_IN))
    X[:, :4] = np.abs(rng.normal(size=(4, 4)))
    _, _, g = N.backward(w, [(X, rng.normal(size=N.N_CTX))], [3.0], quant=False)
    gp = N.unflatten(g)
    assert not gp["W1"].any() and not gp["b1"].any() and not gp["W2"].any()
    assert gp["b4"][0] != 0


def test_huber_closed_forms():
    assert N.huber(0.5) == 0.125
    assert N.huber(-3.0) == 2.5
    assert N.huber_grad(0.25) == 0.25 and N.huber_grad(-7) == -1 and N.huber_grad(7) == 1


def test_adam_first_steps_closed_form():
    st = N.adam_init(3)
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    w1 = N.adam_step(w, g, st, lr=0.01)
    # step 1: m_hat = g, v_hat = g^2 -> update lr * g / (|g| + eps)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    w2 = N.adam_step(w1, g, st, lr=0.01)
    # a constant gradient keeps m_hat = g and v_hat = g^2 exactly
    assert np.allclose(w2, w1 - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    g3 = np.array([0.0, 1.0, 2.0])
    w3 = N.adam_step(w2, g3, st, lr=0.01)
    m = 0.9 * (0.9 * 0.1 * g + 0.1 * g) + 0.1 * g3
    v = 0.999 * (0.999 * 0.001 * g * g + 0.001 * g * g) + 0.001 * g3 * g3
    ref = w2 - 0.01 * (m / (1 - 0.9 ** 3)) / (np.sqrt(v / (1 - 0.999 ** 3)) + 1e-8)
    assert np.allclose(w3, ref, atol=1e-15)


def test_bf16_rounding():
    assert N.bf16(1.0) == 1.0
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties to even keeps 1
    assert N.bf16(1 + 2 ** -8) == 1.0
    assert N.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    assert N.bf16(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7
    assert N.bf16(-3.0) == -3.0
    assert N.bf16(2.0 ** -130) > 0  # float32 subnormals stay representable


def test_features_of_a_tiny_instance():
    """QKP with n = 2: profits [[4, 2], [2, 6]], weights [1, 3], capacity 2."""
    prob = G.Problem(G.KIND_QKP, np.array([[4, 2], [2, 6]]), np.array([[1, 3]]), np.array([2]),
                     Fraction(1))
    par = G.Params(replicas=1, sweeps=2, beta=Fraction(5))
    prog = O.build_program(prob, par)
    fs = N.instance_features(prob, par, prog.n_ext, prog.pq)
    assert len(fs) == 1
    X = fs[0].X
    s_f = 6.0
    assert np.allclose(X[:, 0], [(4 + 2) / (s_f * 2), (6 + 2) / (s_f * 2)])
    assert np.allclose(X[:, 1], [2 * 1 / 2, 2 * 3 / 2])
    assert np.allclose(X[:, 2], X[:, 1])
    assert np.allclose(X[:, 3], [4 / 6, 1.0])
    # efficiencies e = (h + W/2) / a: 5 / 1 and 7 / 3, relative to rho_bar = 3
    assert np.allclose(X[:, 4], [np.log(5 / 3), np.log(7 / 9)])
    assert not X[:, 5:].any()
    # rho_bar = (4 + 1 + 6 + 1) / (1 + 3) = 3; scale = 256 * 3 * s_g / s_f, s_g = 3
    assert abs(fs[0].scale - 256 * 3 * 3 / 6) < 1e-12
    assert prog.n_ext == 4  # two slack bits for b = 2
    # greedy fill of b = 2: item 0 (weight 1) fits, item 1 (weight 3) is the
    # first that does not: e = 7/3 -> 7/9; b / sum a = 2/4; one item of two taken
    assert np.allclose(fs[0].ctx, [np.log(4) / 8, 1.0, prog.pq / 256 / 4, 5 / 50, 1 / 32, 0.0,
                                   7 / 9, 0.5, 0.5])


def test_to_lambda_q_rounds_half_away():
    assert N.to_lambda_q(0.5, 3.0) == 2
    assert N.to_lambda_q(-0.5, 3.0) == -2
    assert N.to_lambda_q(0.25, 2.0) == 1
    assert N.to_lambda_q(-0.125, 2.0) == 0
