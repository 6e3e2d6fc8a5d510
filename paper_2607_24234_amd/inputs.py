"""Seeded synthetic inputs for the quasistatic beam-plasma solver.

This module holds workload descriptions and random draws only -- none of the model's
arithmetic.  Both the GPU path and the CPU oracle consume what it produces, so it imports
neither of them.

Workloads (all in the paper's normalized units: xi, lengths in c/omega_p, tau in
1/omega_p, densities over n_p):

* ``slab``      uniform cold electron beam n_b = 0.01, gamma = 1000, length 20, 32 modes
                k in [0.05, 4], 256 cells, 100 steps of dtau = 50, noise seed 1e-6.
* ``spectral3d`` the same physics on the 512 x 512 (k_x, k_y) grid over |k| <= 6 (only the
                205,859 modes with |k| <= 6 are marched), length 100, 4096 cells, 2000
                steps of dtau = 10, noise seed 1e-6.
* ``batched``   256 instances, n_b log-uniform in [1e-3, 1e-1], gamma log-uniform in
                [10, 1e4], length uniform in [5, 200] with 128 + 8064 (L - 5)/195 cells,
                128 modes k in [0.05, 4], 200 steps of dtau = 10 / (200 sqrt(n_b/gamma)).
"""
from __future__ import annotations

import math

import numpy as np

# seed kinds and flags, mirrored from include/qs.h
SEED_NOISE = 0
SEED_UNIFORM = 1
SEED_FRONT_IMPULSE = 2
SEED_NONE = 4

ELECTRON = (-1.0, 1.0)   # (q, m) in units of (e, m_e)
POSITRON = (1.0, 1.0)


def k_slab(n=32, kmin=0.05, kmax=4.0):
    """Transverse wavenumbers of the slab workload: n values uniform in [kmin, kmax]."""
    return np.linspace(kmin, kmax, n)


def k_grid_3d(n=512, kmax=6.0):
    """Active modes of an n x n (k_x, k_y) grid k = -kmax + i * 2 kmax / n, kept where |k| <= kmax.

    Returns (kx, ky) in row-major (i_x, i_y) order.
    """
    dk = 2.0 * kmax / n
    ax = -kmax + dk * np.arange(n)
    kx, ky = np.meshgrid(ax, ax, indexing="ij")
    keep = kx * kx + ky * ky <= kmax * kmax
    return np.ascontiguousarray(kx[keep]), np.ascontiguousarray(ky[keep])


def slab(n_modes=32, n_xi=256, n_steps=100):
    """Plain slab run: parameters of the small parity workload."""
    return dict(species=[ELECTRON + (0.01,)], gamma=1000.0, length=20.0, n_xi=n_xi,
                kx=k_slab(n_modes), ky=None, d_tau=50.0, n_steps=n_steps,
                seed_kind=SEED_NOISE, seed_amp=1e-6, rng_seed=0)


def spectral3d(n_grid=512, n_xi=4096, n_steps=2000):
    """3D spectral run on the full k grid."""
    kx, ky = k_grid_3d(n_grid)
    return dict(species=[ELECTRON + (0.01,)], gamma=1000.0, length=100.0, n_xi=n_xi,
                kx=kx, ky=ky, d_tau=10.0, n_steps=n_steps,
                seed_kind=SEED_NOISE, seed_amp=1e-6, rng_seed=0)


def batched(n_instances=256, n_modes=128, n_steps=200, seed=0, max_cells=8192):
    """Batched parameter sweep: one dict per instance (draws from numpy's PCG64)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5157]))
    log_nb = rng.uniform(-3.0, -1.0, n_instances)
    log_g = rng.uniform(1.0, 4.0, n_instances)
    length = rng.uniform(5.0, 200.0, n_instances)
    out = []
    for i in range(n_instances):
        nb, g, L = 10.0 ** log_nb[i], 10.0 ** log_g[i], float(length[i])
        n_xi = int(round(128 + (max_cells - 128) * (L - 5.0) / 195.0))
        d_tau = 10.0 / (n_steps * math.sqrt(nb / g))
        out.append(dict(species=[ELECTRON + (nb,)], gamma=g, length=L, n_xi=n_xi,
                        kx=k_slab(n_modes), ky=None, d_tau=d_tau, n_steps=n_steps,
                        seed_kind=SEED_NOISE, seed_amp=1e-6, rng_seed=seed))
    return out


def gaussian_profile(n_xi, length, center, sigma):
    """Gaussian longitudinal profile sampled at the cell centres (peak 1)."""
    h = length / n_xi
    xi = (np.arange(n_xi) + 0.5) * h
    return np.exp(-0.5 * ((xi - center) / sigma) ** 2)


SEED_CENTROID = 3


def finite_width(nx=256, ny=256, n_xi=8192, n_steps=500, length=200.0, box=16.0, sigma_r=0.5,
                 nb=0.05, gamma=2000.0, d_tau=2.0, seed=0):
    """Narrow electron beam on a transverse grid: Gaussian radial profile, flat top in xi,
    seeded by a centroid offset of 1e-3 sigma_r (hosing) plus 1e-6 density noise."""
    return dict(species=[ELECTRON + (nb,)], gamma=gamma, length=length, n_xi=n_xi,
                nx=nx, ny=ny, lx=box, ly=box, sigma_r=sigma_r, d_tau=d_tau, n_steps=n_steps,
                seed_kind=SEED_CENTROID, seed_amp=1e-6, centroid_offset=1e-3 * sigma_r, rng_seed=seed)


def growth_queries(n, seed):
    """Growth-map queries uniform over the box log10 n_b in [-3, -1], log10 gamma in [1, 4],
    k in [0.05, 4], xi in [0, 200], tau in [0, tau_f] (numpy PCG64), as float32 rows
    (ln n_b, ln gamma, k, xi, tau)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x515259]))
    nb = 10.0 ** rng.uniform(-3, -1, n)
    g = 10.0 ** rng.uniform(1, 4, n)
    k = rng.uniform(0.05, 4.0, n)
    xi = rng.uniform(0.0, 200.0, n)
    tau = rng.uniform(0.0, 1.0, n) * 10.0 * np.sqrt(g / nb)
    return np.stack([np.log(nb), np.log(g), k, xi, tau], axis=1).astype(np.float32)
