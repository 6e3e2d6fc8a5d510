"""FP64 CPU oracle of the slowly-varying-envelope (SVEA) variant -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU baseline may import this module.

The paper (Sec. III.B) writes the master equation without its gamma^-2 term in one
transverse Fourier mode as [(d_xi^2 + 1) d_tau^2 - Gamma^2] n_p = delta(xi) delta(tau); with
n_p = N e^{-i xi} it becomes [d_tau^2 (d_xi^2 - 2 i d_xi) - Gamma^2] N = delta delta, and the
envelope approximation (d_xi N << N) drops d_xi^2 N, leaving the first-order equation
    d_tau^2 d_xi N = (i / 2) Gamma^2 N + (i / 2) delta(xi) delta(tau).
This module solves  d_tau^2 d_xi n = a n + delta(xi) delta(tau)  (so that N = (i/2) n for
a = i Gamma^2 / 2) as a first-order system in tau:
    d_tau n = m,   d_tau m = a * integral_0^xi n dxi',
with, after the impulse, n = 0 and m = 1 behind the front (d_xi d_tau n = delta(xi) at
tau = 0+).  Cells j = 0 .. N-1 of width h carry cell values n_j, m_j; the integral at the
cell centre is h sum_{i<j} n_i + (h/2) n_j; classic fourth-order Runge-Kutta in tau.
"""
from __future__ import annotations

import math

import numpy as np


def svea_coefficient(species, gamma_b, k):
    """a = (i/2) Gamma_CFI^2, Gamma_CFI^2 = sum_s q_s^2 n_bs/(m_s gamma_b) k^2/(1+k^2)
    (Eq. CFI_temporal; the same Gamma as in the master equation)."""
    w2 = sum(q * q * nb / (m * gamma_b) for (q, m, nb) in species)
    k = np.asarray(k, np.float64)
    return 0.5j * w2 * k * k / (1.0 + k * k)


def impulse_state(n_modes, n_xi):
    """State right after the impulse: n = 0, m = 1 in every cell (complex, [cell][mode])."""
    return np.zeros((n_xi, n_modes), np.complex128), np.ones((n_xi, n_modes), np.complex128)


def integral(n, h):
    """h sum_{i<j} n_i + (h/2) n_j along the cell axis (axis 0)."""
    return h * (np.cumsum(n, axis=0) - 0.5 * n)


def rates(n, m, a, h):
    return m, a[None, :] * integral(n, h)


def run(a, n_xi, h, dtau, n_steps, n=None, m=None, out_every=1):
    """Advance (n, m) by n_steps RK4 steps.  Returns (ln_abs_n snapshots [n_snap][cell][mode]
    taken before steps 0, out_every, ..., n, m)."""
    a = np.asarray(a, np.complex128).ravel()
    if n is None:
        n, m = impulse_state(len(a), n_xi)
    snaps = []
    for s in range(n_steps):
        if s % out_every == 0:
            with np.errstate(divide="ignore"):
                snaps.append(np.log(np.abs(n)))
        k1n, k1m = rates(n, m, a, h)
        k2n, k2m = rates(n + 0.5 * dtau * k1n, m + 0.5 * dtau * k1m, a, h)
        k3n, k3m = rates(n + 0.5 * dtau * k2n, m + 0.5 * dtau * k2m, a, h)
        k4n, k4m = rates(n + dtau * k3n, m + dtau * k3m, a, h)
        n = n + dtau / 6.0 * (k1n + 2.0 * k2n + 2.0 * k3n + k4n)
        m = m + dtau / 6.0 * (k1m + 2.0 * k2m + 2.0 * k3m + k4m)
    return (np.array(snaps) if snaps else None), n, m


def envelope_exponent(G, tau, xi):
    """Leading growth exponent of |N| quoted in Sec. III.B: (3 sqrt(3) / 4) (G tau)^(2/3) xi^(1/3)."""
    return 3.0 * math.sqrt(3.0) / 4.0 * (G * tau) ** (2.0 / 3.0) * xi ** (1.0 / 3.0)
