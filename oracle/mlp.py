"""FP64 CPU oracle of the growth-map surrogate network -- TEST INFRASTRUCTURE.

Only the test-suite and the benchmark's CPU-baseline leg may import this module; the
product never does, and this module never imports the product.

The network is a plain multilayer perceptron with the exact (erf-based) GELU activation
(Hendrycks and Gimpel, "Gaussian Error Linear Units", 2016): layer widths
dims = [5, 512, 512, 512, 512, 1], y = W5 h4 + b5, h_l = GELU(z_l), z_l = W_l h_{l-1} + b_l,
h0 = x.  Training minimizes the mean squared error with AdamW (Loshchilov and Hutter,
"Decoupled Weight Decay Regularization", 2019: Adam moments with bias correction, weight
decay applied to the weights directly, not through the gradient).

Everything is computed in float64.  With ``rounding="bf16"`` the function also reproduces
the points where the GPU kernels round an operand to bfloat16 before a matrix-core
product (round to nearest, ties to even, from the float32 value):
  * forward: the stored activations h1..h4 and the weights W2..W4 of the three 512x512
    products; the first layer (5 inputs) and the last (1 output) take unrounded operands;
  * backward: the gradient dz_l entering the 512x512 products (dz_l W_l and dz_l^T h_{l-1},
    l = 2..4) and the activations h_{l-1} / weights W_l they meet.
The accumulation itself stays exact (float64) here; the kernels accumulate in float32.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

DIMS = (5, 512, 512, 512, 512, 1)


# ----------------------------------------------------------------------------- rounding
def bf16_round(a):
    """Round to bfloat16 (8 significant bits) via float32, to nearest, ties to even;
    returned as float64.  NaN and infinities pass through."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    bad = ~np.isfinite(f)
    if np.any(bad):
        out = np.where(bad, f.astype(np.float64), out)
    return out


def _rnd(a, rounding):
    return bf16_round(a) if rounding == "bf16" else np.asarray(a, np.float64)


# ----------------------------------------------------------------------------- activation
def gelu(x):
    """x Phi(x) with the standard normal CDF Phi(x) = (1 + erf(x / sqrt 2)) / 2."""
    x = np.asarray(x, np.float64)
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x), phi the standard normal density."""
    x = np.asarray(x, np.float64)
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


# ----------------------------------------------------------------------------- network
def init_params(rng, dims=DIMS):
    """Weights and biases uniform in [-1/sqrt(fan_in), 1/sqrt(fan_in)] from a numpy
    Generator.  Returns a list of (W [out, in], b [out]) float64 pairs."""
    params = []
    for i in range(len(dims) - 1):
        a = 1.0 / math.sqrt(dims[i])
        W = rng.uniform(-a, a, (dims[i + 1], dims[i]))
        b = rng.uniform(-a, a, dims[i + 1])
        params.append((W, b))
    return params


def forward(params, X, rounding=None):
    """Returns (y [M], cache) for inputs X [M, dims[0]]."""
    X = np.asarray(X, np.float64)
    L = len(params)
    hs, zs = [X], []
    h = X
    for l, (W, b) in enumerate(params):
        last = l == L - 1
        if l == 0 or last:
            z = h @ np.asarray(W, np.float64).T + b
        else:
            z = _rnd(h, rounding) @ _rnd(W, rounding).T + b
        zs.append(z)
        if last:
            h = z
        else:
            h = gelu(z)
            if rounding == "bf16":
                h = bf16_round(h)   # stored activations are bfloat16
            hs.append(h)
    return h[:, 0], {"h": hs, "z": zs}


def mse(y, t):
    """Mean squared error (1/M) sum (y - t)^2 and its gradient with respect to y."""
    y = np.asarray(y, np.float64)
    t = np.asarray(t, np.float64)
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / len(d)


def backward(params, cache, dy, rounding=None):
    """Gradients [(dW, db)] of the loss for upstream gradient dy [M] = dLoss/dy."""
    L = len(params)
    hs, zs = cache["h"], cache["z"]
    grads = [None] * L
    dz = np.asarray(dy, np.float64)[:, None]            # last layer: z = y
    for l in range(L - 1, -1, -1):
        W, _ = params[l]
        h_in = hs[l]
        inner = 0 < l < L - 1                            # a 512x512 product
        a = _rnd(dz, rounding) if inner else dz
        hi = _rnd(h_in, rounding) if inner else h_in
        grads[l] = (a.T @ hi, dz.sum(axis=0))
        if l == 0:
            break
        # gradient flowing into h_{l}: dz_l W_l, then through GELU of z_{l-1}
        Wr = _rnd(W, rounding) if inner else np.asarray(W, np.float64)
        dh = a @ Wr
        dz = dh * gelu_grad(zs[l - 1])
    return grads


def loss_and_grads(params, X, T, rounding=None):
    y, cache = forward(params, X, rounding)
    loss, dy = mse(y, T)
    return loss, backward(params, cache, dy, rounding), y


# ----------------------------------------------------------------------------- optimizer
def adamw_init(params):
    return {"t": 0, "m": [(np.zeros_like(W), np.zeros_like(b)) for W, b in params],
            "v": [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]}


def adamw_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.01):
    """One AdamW update (returns new params; state is updated in place):
        m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
        w <- w - lr ( m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps) + wd w )
    applied to weights and biases alike."""
    state["t"] += 1
    t = state["t"]
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    out = []
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (w, g) in enumerate(((W, gW), (b, gb))):
            m = state["m"][i][j] * beta1 + (1.0 - beta1) * g
            v = state["v"][i][j] * beta2 + (1.0 - beta2) * g * g
            mm = list(state["m"][i]); mm[j] = m; state["m"][i] = tuple(mm)
            vv = list(state["v"][i]); vv[j] = v; state["v"][i] = tuple(vv)
            new.append(w - lr * ((m / c1) / (np.sqrt(v / c2) + eps) + weight_decay * w))
        out.append((new[0], new[1]))
    return out
