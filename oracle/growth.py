"""FP64 CPU oracle of the growth-map definitions -- TEST INFRASTRUCTURE.

Only the test-suite may import this module; the product never does.

* The windowed growth of one (mode, snapshot) column, the learned quantity: with
  A_i^2 = |E_i|^2 + |B_i|^2 at cell centres, W = max(1, round(4 pi / h)) cells (two plasma
  wavelengths) and Hann weights w_i = sin^2(pi (i + 1/2) / W), i = 0..W-1, on the cells
  j - i behind and at xi_j,
      G_j = 1/2 ln( sum_{i <= min(j, W-1)} w_i A_{j-i}^2 / S^2  /  sum_{i <= min(j, W-1)} w_i ),
  written out as the plain weighted sum for every j.  (The plasma response oscillates along
  xi; a one-wavelength box average leaves a ripple wherever the envelope grows across the
  window, the Hann weights take it to second order.)
* The query box and its coordinates b (each in [-1, 1] inside the box), which place a query
  in the held-out error table: log10 n_b + 2, (log10 gamma - 2.5)/1.5, (k - 2.025)/1.975,
  xi/100 - 1, 2 tau/tau_f - 1, with tau_f = 10 sqrt(gamma/n_b) (ten e-folds of the
  temporal CFI rate sqrt(n_b/gamma) of Eq. CFI_temporal at large k).
* The network's inputs x, the same five numbers in coordinates that follow the physics:
  log10 n_b + 2, (log10(gamma k) - 2.1505)/2.4515, 2 log10(k/0.05)/log10(80) - 1,
  2 sqrt(xi/200) - 1, 2 sqrt(t/t_max) - 1 with t = Gamma_CFI tau and t_max = 40/sqrt(17)
  (Gamma_CFI tau at k = 4, tau = tau_f).  In these units the continuum answer depends on
  n_b only through the discretization: Gamma_CFI tau, xi, k and gamma k fix it (the
  master equation with tau -> Gamma_CFI tau has the one parameter 1/(gamma k)).
* The closed-form baseline the network's output is added to,
      B = 1/2 ln(kappa^2 (1 + 3 k^2)/2) + J(M(C, F), O),
      C = ln cosh t,  F = 2 (sqrt(1 + t xi) - 1),  O = 3 ((1 + z)^(1/3) - 1),
      z = (3 sqrt(3)/64) t_e^2 xi,  t_e = t (1 + 1/(gamma k)^2)^(1/2),
      J(a, b) = ln(e^a + e^b - 1),  M(a, b) = -ln(e^-a + e^-b - e^-(a+b))
  (for a, b >= 0: J and M are 0 at a = b = 0, J(a, 0) = a, M(a, 0) = 0, and J -> max,
  M -> min once both are large): the wavelength-averaged field level of the extended
  disturbance at tau = 0 (R3 fields of n_p = S (1 - cos xi)), then the temporal CFI growth C
  (Appendix C, K term) held back near the front by F, whose exponent tends to the
  spatiotemporal CFI exponent 2 sqrt(t xi) of Eq. CFI_ST, and overtaken deep in the beam by
  O, whose exponent tends to the spatiotemporal OTSI exponent (3 sqrt(3)/4) t_e^(2/3)
  xi^(1/3) of Eq. OTSI_ST; the longitudinal term raises the OTSI rate from Gamma_CFI to
  (Gamma_CFI^2 + beta^2)^(1/2), beta = Gamma_CFI/(gamma k) (the Laplace form of the
  transverse master equation, Eq. full_master_eq, at s >> beta).  F and O start linearly in
  t xi and t_e^2 xi, like the leading terms of the series sum (t xi)^n/(n!)^2 and
  sum z^n/(n!)^3 whose logarithms have those exponents, so that B is smooth in the inputs
  and equals the field level at tau = 0.
* The error-table bin of box coordinates: 8 equal bins per coordinate, and the plain
  per-bin 99th percentile of held-out errors.
"""
from __future__ import annotations

import math

import numpy as np

T_MAX = 40.0 / math.sqrt(17.0)


def window_cells(h):
    """Cells of the window: two plasma wavelengths, at least one cell."""
    return max(1, int(round(4.0 * math.pi / h)))


def hann_weights(W):
    """w_i = sin^2(pi (i + 1/2) / W), i = 0..W-1 (weight of the cell i behind xi_j)."""
    return np.sin(math.pi * (np.arange(W) + 0.5) / W) ** 2


def windowed_growth(ln_e, ln_b, h, seed_amp):
    """G for one column: ln_e, ln_b arrays over cells (natural logs of |E|, |B|)."""
    ln_e = np.asarray(ln_e, np.float64)
    ln_b = np.asarray(ln_b, np.float64)
    ls = math.log(seed_amp)
    a2 = np.exp(2.0 * (ln_e - ls)) + np.exp(2.0 * (ln_b - ls))
    W = window_cells(h)
    w = hann_weights(W)
    out = np.empty(len(a2))
    for j in range(len(a2)):
        n = min(j + 1, W)
        num = np.sum(w[:n] * a2[j - np.arange(n)])
        out[j] = 0.5 * math.log(num / np.sum(w[:n]))
    return out


def tau_final(nb, gamma):
    return 10.0 * math.sqrt(gamma / nb)


def _split(q):
    q = np.asarray(q, np.float64)
    return np.exp(q[:, 0]), np.exp(q[:, 1]), q[:, 2], q[:, 3], q[:, 4]


def box_coords(q):
    """q [n, 5] = (ln n_b, ln gamma, k, xi, tau) -> b [n, 5], the box coordinates."""
    nb, g, k, xi, tau = _split(q)
    tf = 10.0 * np.sqrt(g / nb)
    return np.stack([np.log10(nb) + 2.0, (np.log10(g) - 2.5) / 1.5, (k - 2.025) / 1.975,
                     xi / 100.0 - 1.0, 2.0 * tau / tf - 1.0], axis=1)


def inside_box(q):
    b = box_coords(q)
    return np.all((b >= -1.0) & (b <= 1.0), axis=1)


def gamma_cfi_tau(q):
    """t = Gamma_CFI tau of a single electron beam, sqrt(n_b/gamma) k/sqrt(1+k^2) tau."""
    nb, g, k, xi, tau = _split(q)
    return np.sqrt(nb / g) * k / np.sqrt(1.0 + k * k) * tau


def features(q):
    """q [n, 5] -> the network inputs x [n, 5] (module docstring); k is floored at 1e-3 and
    xi, t at 0 so that any query has finite inputs."""
    nb, g, k, xi, tau = _split(q)
    kk = np.maximum(k, 1e-3)
    t = np.maximum(gamma_cfi_tau(np.stack([q[:, 0], q[:, 1], kk, xi, tau], 1)), 0.0)
    return np.stack([np.log10(nb) + 2.0,
                     (np.log10(g * kk) - 2.1505) / 2.4515,
                     2.0 * np.log10(kk / 0.05) / math.log10(80.0) - 1.0,
                     2.0 * np.sqrt(np.maximum(xi, 0.0) / 200.0) - 1.0,
                     2.0 * np.sqrt(t / T_MAX) - 1.0], axis=1)


def field_level(k):
    """1/2 ln(kappa^2 (1 + 3 k^2)/2), the baseline's first term."""
    k = np.asarray(k, np.float64)
    kap = 1.0 / (1.0 + k * k)
    return 0.5 * np.log(kap * kap * (1.0 + 3.0 * k * k) / 2.0)


def join_up(a, b):
    """J(a, b) = ln(e^a + e^b - 1)."""
    return np.log(np.exp(a) + np.exp(b) - 1.0)


def join_down(a, b):
    """M(a, b) = -ln(e^-a + e^-b - e^-(a+b))."""
    return -np.log(np.exp(-a) + np.exp(-b) - np.exp(-(a + b)))


def front_growth(t, xi):
    """F = 2 (sqrt(1 + t xi) - 1)."""
    return 2.0 * (np.sqrt(1.0 + t * xi) - 1.0)


def otsi_growth(te, xi):
    """O = 3 ((1 + z)^(1/3) - 1), z = (3 sqrt(3)/64) t_e^2 xi."""
    return 3.0 * (np.cbrt(1.0 + 3.0 * math.sqrt(3.0) / 64.0 * te * te * xi) - 1.0)


def baseline(q):
    """B(q) of the module docstring (k floored at 1e-3, xi and t at 0)."""
    q = np.asarray(q, np.float64)
    nb, g, k, xi, tau = _split(q)
    kk = np.maximum(k, 1e-3)
    xi = np.maximum(xi, 0.0)
    t = np.maximum(gamma_cfi_tau(np.stack([q[:, 0], q[:, 1], kk, xi, tau], 1)), 0.0)
    te = t * np.sqrt(1.0 + 1.0 / (g * kk) ** 2)
    return field_level(kk) + join_up(join_down(np.log(np.cosh(t)), front_growth(t, xi)), otsi_growth(te, xi))


def bin_of(b):
    """Bin of box coordinates b [n, 5]: 8 per coordinate, row-major in coordinate order."""
    c = np.clip(np.floor((np.asarray(b, np.float64) + 1.0) * 4.0).astype(np.int64), 0, 7)
    out = np.zeros(len(c), np.int64)
    for d in range(5):
        out = out * 8 + c[:, d]
    return out


MIN_COUNT = 32


def p99_table(b, err):
    """Per bin of the box coordinates b: the 99th percentile of the bin's n errors, taken as
    the ceil(0.99 n)-th smallest, or -1 when n < 32."""
    bins = bin_of(b)
    err = np.asarray(err, np.float64)
    out = np.full(8 ** 5, -1.0)
    for bb in np.unique(bins):
        e = np.sort(err[bins == bb])
        if len(e) < MIN_COUNT:
            continue
        out[bb] = e[int(math.ceil(0.99 * len(e))) - 1]
    return out
