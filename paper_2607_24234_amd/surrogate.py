"""Growth-map surrogate pipeline: training data from batched solver runs, training, held-out
error table, and queries.  Every step runs in the library's kernels (libqs); this module
only orders the calls and owns the torch buffers.

Training data: the batched sweep of the inputs module (log-uniform n_b in [1e-3, 1e-1],
gamma in [10, 1e4], L in [5, 200], 128 modes k in [0.05, 4], d_tau = tau_f/200) seeded with
the uniform extended disturbance, snapshots of ln|E|, ln|B| every `snap_every` steps up to
tau_f, the windowed growth G of each entry (include/qs_growth.h), and examples drawn
uniformly over (snapshot, instance, cell, mode).  A second sweep with its own parameter
draws is held out: its examples measure the network's error and fill the error table that
routes queries.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs, qs


def sweep_instances(n_instances=256, n_modes=128, n_steps=200, seed=0, max_cells=8192):
    insts = inputs.batched(n_instances=n_instances, n_modes=n_modes, n_steps=n_steps, seed=seed,
                           max_cells=max_cells)
    for d in insts:
        d["seed_kind"] = inputs.SEED_UNIFORM
    return insts


def examples(insts, n_samples, sample_seed, n_steps=200, snap_every=10, device="cuda"):
    """Run the solver over `insts` (FP32 state), compute G on every snapshot and draw
    n_samples examples.  Returns (X [n, 5], T [n]) torch tensors on the device."""
    import torch
    s = qs.Solver(insts, precision=qs.QS_FP32)
    out = s.step(n_steps, out_every=snap_every, snapshots=True)
    fin = s.step(0, snapshots=True)
    s.sync_check()
    ln_e = torch.cat([out["ln_e"], fin["ln_e"]])
    ln_b = torch.cat([out["ln_b"], fin["ln_b"]])
    del out, fin
    steps = np.array(list(range(0, n_steps, snap_every)) + [n_steps], np.int32)
    gi = qs.GrowthInstances(insts)
    G = torch.empty_like(ln_e)
    qs.growth_targets(gi, ln_e, ln_b, G, stream=s.stream)
    del ln_e, ln_b
    X = torch.empty((n_samples, 5), dtype=torch.float32, device=device)
    T = torch.empty(n_samples, dtype=torch.float32, device=device)
    qs.growth_sample(gi, G, steps, sample_seed, n_samples, X, T, stream=s.stream)
    torch.cuda.synchronize()
    s.close()
    return X, T


def split(insts, every=10):
    train = [d for i, d in enumerate(insts) if i % every != every - 1]
    held = [d for i, d in enumerate(insts) if i % every == every - 1]
    return train, held


def initial_params(seed=0, out_mean=0.0, out_scale=1.0):
    """Weights and biases uniform in [-1/sqrt(fan_in), 1/sqrt(fan_in)] (numpy PCG64); the
    output layer scaled by out_scale with bias out_mean, so that the initial outputs have
    the targets' centre and spread."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x4D4C50]))
    dims = qs.MLP_DIMS
    P = [(rng.uniform(-1 / math.sqrt(dims[i]), 1 / math.sqrt(dims[i]), (dims[i + 1], dims[i])),
          rng.uniform(-1 / math.sqrt(dims[i]), 1 / math.sqrt(dims[i]), dims[i + 1])) for i in range(len(dims) - 1)]
    W5, _ = P[-1]
    P[-1] = (W5 * out_scale, np.array([out_mean]))
    return P


def train(net, X, T, epochs=20, batch=8192, lr=1e-3, lr_min=1e-5, log=None):
    """AdamW (weight decay 0.01) over contiguous batches of the (already random) examples,
    cosine learning-rate decay from lr to lr_min.  Returns the mean loss of the last epoch."""
    n = (X.shape[0] // batch) * batch
    steps = n // batch
    total = epochs * steps
    k = 0
    last = float("nan")
    for ep in range(epochs):
        acc = 0.0
        shift = (ep * 7919) % steps        # a different batch order each epoch
        for i in range(steps):
            b = (i + shift) % steps
            t = k / max(1, total - 1)
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * t))
            want = i == steps - 1
            l = net.train_step(X[b * batch:(b + 1) * batch], T[b * batch:(b + 1) * batch], lr_t, want_loss=want)
            if want:
                acc = l
            k += 1
        last = acc
        if log:
            log("epoch %d loss %.3e lr %.2e" % (ep, acc, lr_t))
    return last


def held_out_errors(net, X, T):
    import torch
    y = net.forward(X)
    e = (y - T).abs()
    torch.cuda.synchronize()
    ec = e.cpu().numpy()
    return {"rms": float(np.sqrt(np.mean(ec ** 2))), "p50": float(np.percentile(ec, 50)),
            "p99": float(np.percentile(ec, 99)), "max": float(ec.max()),
            "frac_le_1e-2": float(np.mean(ec <= 1e-2))}


def calibrate(net, X, T):
    import torch
    table = torch.empty(qs.GROWTH_BINS, dtype=torch.float32, device=X.device)
    qs.growth_calibrate(net, X, T, table)
    return table


def save(path, net, table, meta):
    np.savez(path, params=net.get_params(), table=table.cpu().numpy(), meta=np.array(repr(meta)))


def load(path, max_batch=65536):
    import torch
    d = np.load(path, allow_pickle=False)
    net = qs.MLP(max_batch=max_batch)
    net.set_params(d["params"])
    return net, torch.as_tensor(d["table"], device="cuda")


def query_box(n, seed):
    """Queries uniform over (log n_b, log gamma, k, xi in [0, 200], tau in [0, tau_f])
    (numpy PCG64), as float32 rows (ln n_b, ln gamma, k, xi, tau)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x515259]))
    nb = 10.0 ** rng.uniform(-3, -1, n)
    g = 10.0 ** rng.uniform(1, 4, n)
    k = rng.uniform(0.05, 4.0, n)
    xi = rng.uniform(0.0, 200.0, n)
    tau = rng.uniform(0.0, 1.0, n) * 10.0 * np.sqrt(g / nb)
    return np.stack([np.log(nb), np.log(g), k, xi, tau], axis=1).astype(np.float32)
