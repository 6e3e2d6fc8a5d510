"""GPU parity of the surrogate network kernels (include/qs_mlp.h) against the FP64 oracle
(oracle/mlp.py) evaluated with the same bfloat16 rounding points.

What remains between the two is float32 accumulation (K = 512 terms, relative ~2^-24 sqrt K
of the sum of |terms|) and, rarely, a stored bfloat16 activation that lands on the other
side of a rounding boundary (one bfloat16 unit, 2^-8 relative, of one element).  The
tolerances below are written from those two effects.
"""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = M.init_params(rng)
    return [(W * scale, b * scale) for W, b in P]


def _as_f32(P):
    return [(np.float32(W).astype(np.float64), np.float32(b).astype(np.float64)) for W, b in P]


def _row_scale(P, cache):
    """sum_o |w5_o h4_o| + |b5| per row: the magnitude the last layer adds up."""
    W5, b5 = P[-1]
    return np.abs(cache["h"][-1]) @ np.abs(W5[0]) + abs(b5[0])


@pytest.mark.parametrize("n", [1, 127, 1000, 4096 + 77])
def test_forward_matches_oracle(qs, n):
    import torch
    P = _as_f32(_params(1))
    X = np.random.default_rng(2).uniform(-1.5, 1.5, (n, 5)).astype(np.float32)
    net = qs.MLP(max_batch=1024)   # several chunks plus a ragged one for the larger n
    net.set_params(qs.pack_params(P))
    y = net.forward(torch.as_tensor(X, device="cuda")).cpu().numpy().astype(np.float64)
    ref, cache = M.forward(P, X.astype(np.float64), rounding="bf16")
    scale = _row_scale(P, cache)
    err = np.abs(y - ref)
    # one bfloat16 unit of the row's magnitude bounds a boundary crossing; typical rows
    # differ only by float32 accumulation
    assert np.all(err <= 2.0 ** -8 * scale), float(np.max(err / scale))
    assert np.median(err / scale) <= 1e-5, float(np.median(err / scale))


def test_forward_beyond_one_launch(qs):
    """2^25 + 77 queries: two launches of the persistent inference kernel (2^25 queries per
    launch) and a ragged last tile; sampled rows at both ends and across the launch boundary
    against the oracle."""
    import torch
    P = _as_f32(_params(11))
    n = (1 << 25) + 77
    g = torch.Generator(device="cuda").manual_seed(12)
    X = (torch.rand((n, 5), device="cuda", generator=g) * 3.0 - 1.5).contiguous()
    net = qs.MLP(max_batch=128)
    net.set_params(qs.pack_params(P))
    y = net.forward(X)
    torch.cuda.synchronize()
    rows = np.concatenate([np.arange(300), np.arange((1 << 25) - 300, (1 << 25) + 77),
                           np.random.default_rng(13).choice(n, 1000, replace=False)])
    xs = X[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    ys = y[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    ref, cache = M.forward(P, xs, rounding="bf16")
    scale = _row_scale(P, cache)
    err = np.abs(ys - ref)
    assert np.all(err <= 2.0 ** -8 * scale), float(np.max(err / scale))
    assert np.median(err / scale) <= 1e-5


def test_gradients_match_oracle(qs):
    import torch
    P = _as_f32(_params(3))
    rng = np.random.default_rng(4)
    B = 1024
    X = rng.uniform(-1.5, 1.5, (B, 5)).astype(np.float32)
    T = rng.standard_normal(B).astype(np.float32)
    net = qs.MLP(max_batch=2048)
    net.set_params(qs.pack_params(P))
    loss = net.grads(torch.as_tensor(X, device="cuda"), torch.as_tensor(T, device="cuda"))
    G = qs.unpack_params(net.get_grads())
    rl, RG, _ = M.loss_and_grads(P, X.astype(np.float64), T.astype(np.float64), rounding="bf16")
    assert abs(loss - rl) <= 1e-5 * rl
    names = ["W1", "W2", "W3", "W4", "W5"]
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(G, RG)):
        for g, r, what in ((gW, rW, names[l]), (gb, rb, "b%d" % (l + 1))):
            e = np.abs(g - r)
            s = np.max(np.abs(r))
            # each gradient is a sum over the batch of products of bfloat16 operands: a
            # flipped operand moves it by at most 2^-8 of one term; accumulation order by
            # ~2^-24 sqrt(B) of the sum of |terms|
            assert np.max(e) <= 2.0 ** -8 * s, (what, float(np.max(e) / s))
            assert np.median(e) <= 1e-4 * s, (what, float(np.median(e) / s))


def test_gradients_deterministic(qs):
    import torch
    P = _as_f32(_params(5))
    rng = np.random.default_rng(6)
    X = torch.as_tensor(rng.uniform(-1, 1, (2048, 5)).astype(np.float32), device="cuda")
    T = torch.as_tensor(rng.standard_normal(2048).astype(np.float32), device="cuda")
    out = []
    for _ in range(2):
        net = qs.MLP(max_batch=2048)
        net.set_params(qs.pack_params(P))
        net.grads(X, T)
        out.append(net.get_grads())
    assert np.array_equal(out[0], out[1])


def test_adamw_matches_oracle(qs):
    """Gradients drawn here go into both optimizers; three steps."""
    P = _as_f32(_params(7))
    rng = np.random.default_rng(8)
    net = qs.MLP(max_batch=128)
    net.set_params(qs.pack_params(P))
    st = M.adamw_init(P)
    Q = P
    for step in range(3):
        G = [(np.float32(rng.standard_normal(W.shape) * 1e-2).astype(np.float64),
              np.float32(rng.standard_normal(b.shape) * 1e-2).astype(np.float64)) for W, b in P]
        net.set_grads(qs.pack_params(G))
        net.adamw(1e-3, 0.9, 0.999, 1e-8, 0.01)
        Q = M.adamw_step(Q, G, st, 1e-3, 0.9, 0.999, 1e-8, 0.01)
    got = qs.unpack_params(net.get_params())
    for (gW, gb), (rW, rb), (W0, b0) in zip(got, Q, P):
        # float32 arithmetic on an update of size ~lr: relative 1e-5 of lr plus one float32
        # rounding of the weight
        assert np.max(np.abs(gW - rW) - 2.0 ** -23 * np.abs(rW)) <= 1e-5 * 1e-3 * 3
        assert np.max(np.abs(gb - rb) - 2.0 ** -23 * np.abs(rb)) <= 1e-5 * 1e-3 * 3


def test_training_steps_track_oracle(qs):
    """Five AdamW steps on the same batch from the same start: losses agree."""
    import torch
    P = _as_f32(_params(9))
    rng = np.random.default_rng(10)
    B = 512
    X = rng.uniform(-1, 1, (B, 5)).astype(np.float32)
    T = (np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 3]).astype(np.float32)
    net = qs.MLP(max_batch=B)
    net.set_params(qs.pack_params(P))
    xd, td = torch.as_tensor(X, device="cuda"), torch.as_tensor(T, device="cuda")
    st = M.adamw_init(P)
    Q = P
    for step in range(5):
        gl = net.train_step(xd, td, 1e-3, want_loss=True)
        rl, RG, _ = M.loss_and_grads(Q, X.astype(np.float64), T.astype(np.float64), rounding="bf16")
        Q = M.adamw_step(Q, RG, st, 1e-3)
        assert abs(gl - rl) <= 2e-3 * rl, (step, gl, rl)
    assert rl < M.loss_and_grads(P, X.astype(np.float64), T.astype(np.float64), rounding="bf16")[0]


def test_argument_errors(qs):
    import ctypes
    L = qs.lib()
    h = ctypes.c_void_p()
    assert L.qs_mlp_create(100, None, ctypes.byref(h)) == qs.QS_ERR_ARG
    assert L.qs_mlp_create(0, None, ctypes.byref(h)) == qs.QS_ERR_ARG
    net = qs.MLP(max_batch=256)
    import torch
    x = torch.zeros((512, 5), device="cuda")
    t = torch.zeros(512, device="cuda")
    with pytest.raises(qs.QSError):
        net.grads(x, t)           # batch above max_batch
    with pytest.raises(qs.QSError):
        net.grads(x[:100], t[:100])   # not a multiple of 128
