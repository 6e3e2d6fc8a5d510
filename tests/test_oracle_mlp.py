"""Pins of the surrogate network's oracle (oracle/mlp.py) against values fixed by
mathematics: the normal CDF, bfloat16's definition, a network small enough to write out by
hand, central finite differences, and AdamW's first step in closed form."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_values():
    # Phi(1) = 0.8413447460685429..., Phi(-1) = 1 - Phi(1); GELU(x) - GELU(-x) = x
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(-1.0) + (1 - 0.8413447460685429)) < 1e-15
    x = np.linspace(-6, 6, 101)
    assert np.max(np.abs(mlp.gelu(x) - mlp.gelu(-x) - x)) < 1e-14
    assert mlp.gelu(0.0) == 0.0
    # large arguments: GELU(x) -> x, GELU(-x) -> 0
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-12 and abs(mlp.gelu(-10.0)) < 1e-12


def test_gelu_grad_against_differences():
    x = np.linspace(-5, 5, 41)
    e = 1e-6
    fd = (mlp.gelu(x + e) - mlp.gelu(x - e)) / (2 * e)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8
    # phi(0) = 1/sqrt(2 pi): GELU'(0) = 1/2
    assert abs(mlp.gelu_grad(0.0) - 0.5) < 1e-16


def test_bf16_rounding_definition():
    r = mlp.bf16_round
    assert r(1.0) == 1.0
    assert r(1 + 2.0 ** -8) == 1.0                     # halfway: ties to even
    assert r(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6       # halfway: ties to even (upwards)
    assert r(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7
    assert r(-3.14159265) == -3.140625
    assert r(0.0) == 0.0 and np.isnan(r(np.nan)) and r(np.inf) == np.inf
    # 8 significant bits: every bf16 value is a fixed point, and the relative error of
    # rounding to nearest is at most the unit roundoff 2^-8
    x = np.random.default_rng(1).standard_normal(10000) * 100
    y = r(x)
    assert np.array_equal(r(y), y)
    assert np.max(np.abs(y - x) / np.abs(x)) <= 2.0 ** -8
    assert np.max(np.abs(y - x) / np.abs(x)) > 0.9 * 2.0 ** -8   # attained: not truncation-free


def test_forward_by_hand():
    """dims [2, 1, 1]: y = w2 GELU(w1 . x + b1) + b2."""
    P = [(np.array([[0.5, -1.5]]), np.array([0.25])), (np.array([[2.0]]), np.array([-1.0]))]
    X = np.array([[1.0, 0.0], [0.0, 1.0], [2.0, 3.0]])
    y, cache = mlp.forward(P, X)
    for i, (a, b) in enumerate(X):
        z = 0.5 * a - 1.5 * b + 0.25
        ref = 2.0 * (0.5 * z * (1 + math.erf(z / math.sqrt(2)))) - 1.0
        assert abs(y[i] - ref) < 1e-15


def test_gradients_against_central_differences():
    rng = np.random.default_rng(7)
    dims = (5, 7, 6, 5, 4, 1)
    P = mlp.init_params(rng, dims)
    X = rng.standard_normal((13, 5))
    T = rng.standard_normal(13)
    loss, G, _ = mlp.loss_and_grads(P, X, T)
    e = 1e-6
    for l in range(len(P)):
        W, b = P[l]
        for idx in [(0, 0), (W.shape[0] - 1, W.shape[1] - 1), (W.shape[0] // 2, W.shape[1] // 2)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += e
            Wm[idx] -= e
            lp = mlp.loss_and_grads(P[:l] + [(Wp, b)] + P[l + 1:], X, T)[0]
            lm = mlp.loss_and_grads(P[:l] + [(Wm, b)] + P[l + 1:], X, T)[0]
            fd = (lp - lm) / (2 * e)
            assert abs(fd - G[l][0][idx]) <= 1e-7 * max(1.0, abs(fd)), (l, idx)
        for k in (0, len(b) - 1):
            bp, bm = b.copy(), b.copy()
            bp[k] += e
            bm[k] -= e
            lp = mlp.loss_and_grads(P[:l] + [(W, bp)] + P[l + 1:], X, T)[0]
            lm = mlp.loss_and_grads(P[:l] + [(W, bm)] + P[l + 1:], X, T)[0]
            fd = (lp - lm) / (2 * e)
            assert abs(fd - G[l][1][k]) <= 1e-7 * max(1.0, abs(fd)), (l, k)


def test_rounded_gradients_equal_exact_on_bf16_inputs():
    """With every rounded quantity already a bfloat16 value, rounding changes nothing: the
    emulated-rounding path must then equal the exact path (catches a rounding applied to
    the wrong operand only in combination with the next test)."""
    rng = np.random.default_rng(3)
    dims = (5, 8, 8, 8, 8, 1)
    P = [(mlp.bf16_round(W), b) for W, b in mlp.init_params(rng, dims)]
    X = rng.standard_normal((6, 5))
    y0, c0 = mlp.forward(P, X)
    y1, c1 = mlp.forward(P, X, rounding="bf16")
    # activations are rounded when stored, so only those differ: bounded by the rounding
    for h0, h1 in zip(c0["h"][1:], c1["h"][1:]):
        assert np.max(np.abs(h1 - mlp.bf16_round(h0))) <= 2.0 ** -7 * np.max(np.abs(h0))
    assert np.max(np.abs(y1 - y0)) < 0.05 * np.max(np.abs(y0)) + 1e-3


def test_rounding_points():
    """Rounding the first layer's or last layer's operands would change these outputs; the
    inner products' operands are rounded: checked by perturbing inputs below bf16
    resolution (invisible to rounded operands, visible to unrounded ones)."""
    rng = np.random.default_rng(5)
    dims = (5, 4, 4, 4, 4, 1)
    P = mlp.init_params(rng, dims)
    X = rng.standard_normal((3, 5))
    y, _ = mlp.forward(P, X, rounding="bf16")
    # the first layer takes unrounded inputs: a tiny input change moves z1
    _, c = mlp.forward(P, X + 1e-9, rounding="bf16")
    _, c0 = mlp.forward(P, X, rounding="bf16")
    assert np.any(c["z"][0] != c0["z"][0])
    # an inner weight perturbed far below bf16 resolution leaves the output unchanged
    P2 = list(P)
    W2, b2 = P[1]
    P2[1] = (mlp.bf16_round(W2) * (1 + 1e-12), b2)
    P1 = list(P)
    P1[1] = (mlp.bf16_round(W2), b2)
    assert np.array_equal(mlp.forward(P1, X, rounding="bf16")[0], mlp.forward(P2, X, rounding="bf16")[0])
    # ... but the last layer's weights are not rounded
    P3 = list(P)
    W5, b5 = P[4]
    P3[4] = (W5 * (1 + 1e-12), b5)
    assert not np.array_equal(mlp.forward(P3, X, rounding="bf16")[0], y)


def test_adamw_first_step_closed_form():
    """t = 1 from zero moments: m/(1-b1) = g and v/(1-b2) = g^2, so the step is
    w - lr (g/(|g| + eps) + wd w)."""
    rng = np.random.default_rng(11)
    P = mlp.init_params(rng, (5, 3, 2, 2, 2, 1))
    G = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in P]
    st = mlp.adamw_init(P)
    lr, wd, eps = 1e-3, 0.01, 1e-8
    Q = mlp.adamw_step(P, G, st, lr, eps=eps, weight_decay=wd)
    for (W, b), (gW, gb), (W1, b1) in zip(P, G, Q):
        assert np.allclose(W1, W - lr * (gW / (np.abs(gW) + eps) + wd * W), rtol=0, atol=1e-15)
        assert np.allclose(b1, b - lr * (gb / (np.abs(gb) + eps) + wd * b), rtol=0, atol=1e-15)
    # second step with the same gradient: m = g(1-b1^2)... bias-corrected m/c1 = g again,
    # v/c2 = g^2 again, so the step has the same form
    Q2 = mlp.adamw_step(Q, G, st, lr, eps=eps, weight_decay=wd)
    for (W, b), (gW, gb), (W2, b2) in zip(Q, G, Q2):
        assert np.allclose(W2, W - lr * (gW / (np.abs(gW) + eps) + wd * W), rtol=0, atol=1e-14)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    dims = (5, 16, 16, 16, 16, 1)
    P = mlp.init_params(rng, dims)
    X = rng.uniform(-1, 1, (256, 5))
    T = np.sin(X[:, 0]) + X[:, 1] * X[:, 2]
    st = mlp.adamw_init(P)
    l0 = mlp.loss_and_grads(P, X, T)[0]
    for _ in range(200):
        _, G, _ = mlp.loss_and_grads(P, X, T)
        P = mlp.adamw_step(P, G, st, 3e-3)
    assert mlp.loss_and_grads(P, X, T)[0] < 0.2 * l0


def test_rounded_backward_within_rounding_bound():
    """The emulated-rounding gradients differ from the exact gradients of the same rounded
    forward only by the bf16 rounding of the products' operands (relative 2^-8 each): a
    misplaced transpose or a dropped term in the rounded branch would exceed this bound."""
    rng = np.random.default_rng(9)
    dims = (5, 32, 32, 32, 32, 1)
    P = mlp.init_params(rng, dims)
    X = rng.standard_normal((40, 5))
    T = rng.standard_normal(40)
    y, cache = mlp.forward(P, X, rounding="bf16")
    _, dy = mlp.mse(y, T)
    g_r = mlp.backward(P, cache, dy, rounding="bf16")
    g_x = mlp.backward(P, cache, dy, rounding=None)
    for (dWr, dbr), (dWx, dbx) in zip(g_r, g_x):
        scale = np.max(np.abs(dWx)) + 1e-300
        assert np.max(np.abs(dWr - dWx)) <= 2.0 ** -5 * scale
        assert np.max(np.abs(dbr - dbx)) <= 2.0 ** -5 * (np.max(np.abs(dbx)) + 1e-300)
