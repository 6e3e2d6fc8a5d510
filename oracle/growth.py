"""FP64 CPU oracle of the growth-map definitions -- TEST INFRASTRUCTURE.

Only the test-suite may import this module; the product never does.

* The windowed growth of one (mode, snapshot) column: with A_i^2 = |E_i|^2 + |B_i|^2 at
  cell centres and w = max(1, round(2 pi / h)) cells per plasma wavelength,
      G_j = 1/2 ln( (1 / c_j) sum_{i = j - c_j + 1}^{j} A_i^2 / S^2 ),  c_j = min(j + 1, w),
  written out as the plain sum for every j.
* The feature map of a query (ln n_b, ln gamma, k, xi, tau) onto [-1, 1]^5 and the final
  time tau_f = 10 sqrt(gamma / n_b) of the batched sweep (ten e-folds of the temporal CFI
  rate sqrt(n_b / gamma) of Eq. CFI_temporal at large k).
* The error-table bin of a feature vector: 8 equal bins per feature over [-1, 1].
"""
from __future__ import annotations

import math

import numpy as np


def window_cells(h):
    return max(1, int(round(2.0 * math.pi / h)))


def windowed_growth(ln_e, ln_b, h, seed_amp):
    """G for one column: ln_e, ln_b arrays over cells (natural logs of |E|, |B|)."""
    ln_e = np.asarray(ln_e, np.float64)
    ln_b = np.asarray(ln_b, np.float64)
    ls = math.log(seed_amp)
    a2 = np.exp(2.0 * (ln_e - ls)) + np.exp(2.0 * (ln_b - ls))
    w = window_cells(h)
    out = np.empty(len(a2))
    for j in range(len(a2)):
        lo = max(0, j - w + 1)
        out[j] = 0.5 * math.log(np.sum(a2[lo:j + 1]) / (j + 1 - lo))
    return out


def tau_final(nb, gamma):
    return 10.0 * math.sqrt(gamma / nb)


def features(q):
    """q [n, 5] = (ln n_b, ln gamma, k, xi, tau) -> x [n, 5]."""
    q = np.asarray(q, np.float64)
    nb, g = np.exp(q[:, 0]), np.exp(q[:, 1])
    tf = 10.0 * np.sqrt(g / nb)
    return np.stack([np.log10(nb) + 2.0, (np.log10(g) - 2.5) / 1.5, (q[:, 2] - 2.025) / 1.975,
                     q[:, 3] / 100.0 - 1.0, 2.0 * q[:, 4] / tf - 1.0], axis=1)


def bin_of(x):
    c = np.clip(np.floor((np.asarray(x, np.float64) + 1.0) * 4.0).astype(np.int64), 0, 7)
    b = np.zeros(len(c), np.int64)
    for d in range(5):
        b = b * 8 + c[:, d]
    return b


E0 = 1e-4
BUCKETS = 64
MIN_COUNT = 32


def bucket(e):
    """Histogram bucket of an error: 0 for e <= 1e-4, else 1 + floor(4 log2(e / 1e-4)),
    at most 63 (also for non-finite errors)."""
    e = float(e)
    if not (e <= 3.0e38):
        return BUCKETS - 1
    if e <= E0:
        return 0
    return min(BUCKETS - 1, 1 + int(math.floor(4.0 * math.log2(e / E0))))


def bucket_edge(b):
    return 3.0e38 if b >= BUCKETS - 1 else E0 * 2.0 ** (0.25 * b)


def p99_table(x, err):
    """Per bin: the upper edge of the bucket holding the ceil(0.99 n)-th smallest error of the
    bin's n examples, or -1 when n < 32."""
    bins = bin_of(x)
    out = np.full(8 ** 5, -1.0)
    for b in np.unique(bins):
        e = np.asarray(err)[bins == b]
        if len(e) < MIN_COUNT:
            continue
        k = int(math.ceil(0.99 * len(e)))
        counts = np.bincount([bucket(v) for v in e], minlength=BUCKETS)
        acc = np.cumsum(counts)
        out[b] = bucket_edge(int(np.argmax(acc >= k)))
    return out
