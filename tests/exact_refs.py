"""Exact and asymptotic references taken from the paper (test-only, independent of oracle/).

Every function cites the passage it restates.  Nothing here calls the oracle or the GPU
path; these are the values the oracle is pinned to.
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np


def gamma_cfi(species, gamma_b, k):
    """Temporal CFI rate, Eq. CFI_temporal: (sum_s omega_bs^2 k^2/(k^2+1))^(1/2) with
    omega_bs^2 = q_s^2 n_bs/(m_s gamma_b) (definition below Eq. full_master_eq)."""
    w2 = sum(q * q * nb / (m * gamma_b) for (q, m, nb) in species)
    return math.sqrt(w2 * k * k / (k * k + 1.0))


def gamma_otsi(species, gamma_b, k):
    """Temporal OTSI rate, Eq. OTSI_temporal."""
    w2 = sum(q * q * nb / (m * gamma_b) for (q, m, nb) in species)
    return math.sqrt(3.0) / 2 ** (4.0 / 3.0) * w2 ** (1.0 / 3.0) * \
        ((k * k + gamma_b ** -2) / (k * k + 1.0)) ** (1.0 / 3.0)


def gamma_tsi(species, gamma_b):
    """Temporal TSI rate (Sec. IV.A): sqrt(3)/2^(4/3) (sum_s omega_bs^2/gamma_b^2)^(1/3)."""
    w2 = sum(q * q * nb / (m * gamma_b) for (q, m, nb) in species)
    return math.sqrt(3.0) / 2 ** (4.0 / 3.0) * (w2 / gamma_b ** 2) ** (1.0 / 3.0)


def rk4_growth_factor(z):
    """Amplification factor of classic RK4 for y' = lambda y with z = lambda dt."""
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def impulse_series(tau, xi, G, dps=40, tol=1e-30):
    """Exact impulse response of [(d_xi^2+1) d_tau^2 - G^2] n = delta(xi) delta(tau)
    (Eq. CFI_st_master with a delta source).  Laplace-transforming in tau gives
    n = sin(kappa xi)/(kappa s^2), kappa^2 = 1 - G^2/s^2 (Eq. n_alpha_xi with alpha = -i s);
    expanding in G^2/s^2 with spherical Bessel functions and inverting term by term:
        n = sum_j G^(2j) tau^(2j+1)/(2j+1)! * xi^(j+1) j_j(xi) / (2^j j!).
    The j = 0 term, tau sin(xi), is the free plasma response."""
    if xi <= 0 or tau <= 0:
        return 0.0
    with mp.workdps(dps):
        G, tau, xi = mp.mpf(G), mp.mpf(tau), mp.mpf(xi)
        total = mp.mpf(0)
        j = 0
        big = mp.mpf(0)
        while True:
            jj = mp.sqrt(mp.pi / (2 * xi)) * mp.besselj(j + mp.mpf(1) / 2, xi)
            term = G ** (2 * j) * tau ** (2 * j + 1) / mp.factorial(2 * j + 1) * \
                xi ** (j + 1) * jj / (2 ** j * mp.factorial(j))
            total += term
            big = max(big, abs(term))
            if j > 4 and abs(term) < tol * max(big, mp.mpf(1e-300)) and j > xi:
                break
            j += 1
            if j > 4000:
                raise RuntimeError("impulse series did not converge")
        return float(total)


def front_limit_exact(tau, xi, G):
    """Exact impulse response of (d_tau^2 d_xi^2 - G^2) n = delta(xi) delta(tau),
    Eq. CFI_st_master_front, solved in Appendix A:  [I_0(2 sqrt(G xi tau)) - J_0(...)]/(2G)."""
    if xi <= 0 or tau <= 0:
        return 0.0
    z = 2.0 * math.sqrt(G * xi * tau)
    return float((mp.besseli(0, z) - mp.besselj(0, z)) / (2.0 * G))


def asym_front(tau, xi, G):
    """Front-region asymptote, Eq. CFI_ST / Eq. np_small_C (xi << xi_tr)."""
    th = xi / tau
    return (1 + 3 * th / (8 * G)) / (4 * math.sqrt(math.pi)) * \
        math.exp(2 * math.sqrt(G * tau * xi) * (1 - th / (4 * G))) / (G * (G * tau * xi) ** 0.25)


def asym_critical(tau, G):
    """Critical-line asymptote, Eq. CFI_T / Eq. np_C_cr, at xi = (2/sqrt(27)) G tau."""
    return 3 ** (1.0 / 6.0) * math.gamma(1.0 / 3.0) * math.exp(4.0 / 3.0 * math.sqrt(2.0 / 3.0) * G * tau) / \
        (4 * math.sqrt(2.0) * math.pi * G * (G * tau) ** (1.0 / 3.0))


def asym_rear(tau, xi, G):
    """Rear asymptote (spatiotemporal OTSI), Eq. OTSI_ST / Eq. np_large_C; returns the real
    value 2 Re{...}."""
    C = xi / (G * tau)
    pref = 1.0 / (4 * G) * math.sqrt(2.0 / (3 * math.pi * xi))
    corr = 1 + 1.0 / (6 * C ** (2.0 / 3.0)) * complex(0.25, math.sqrt(3) / 2)
    ph = 1j * xi + 0.75 * complex(math.sqrt(3), -1) * (G * tau) ** (2.0 / 3.0) * xi ** (1.0 / 3.0) - 1j * math.pi / 4
    return pref * 2 * (corr * np.exp(ph)).real


def xi_transition(G, tau):
    """CFI/OTSI transition point xi_tr = (2/sqrt(27)) G tau (Sec. III.B)."""
    return 2.0 / math.sqrt(27.0) * G * tau


def impulse_series_long(tau, xi, G, beta, dps=40, tol=1e-30):
    """Exact impulse response of the transverse master equation with its longitudinal term,
    [(d_xi^2+1) d_tau^2 - G^2 + beta^2 d_xi^2] n = delta(xi) delta(tau)  (Eq. full_master_eq in
    one Fourier mode: G^2 = sum w^2 k^2/(1+k^2), beta^2 = sum w^2/(gamma^2 (1+k^2))).

    Laplace in tau: n = sin(kappa xi)/(kappa (s^2+beta^2)), kappa^2 = (s^2-G^2)/(s^2+beta^2).
    With 1 - kappa^2 = (G^2+beta^2)/(s^2+beta^2) and the spherical-Bessel expansion of
    sin(xi sqrt(q))/sqrt(q) about q = 1,
        n(s) = sum_j xi^(j+1) j_j(xi)/(2^j j!) (G^2+beta^2)^j / (s^2+beta^2)^(j+1),
    and L^-1[(s^2+b^2)^-m] = sqrt(pi)/Gamma(m) (tau/2b)^(m-1/2) J_(m-1/2)(b tau).
    For beta -> 0 this is impulse_series."""
    if xi <= 0 or tau <= 0:
        return 0.0
    if beta == 0:
        return impulse_series(tau, xi, G, dps, tol)
    with mp.workdps(dps):
        G, b, tau, xi = mp.mpf(G), mp.mpf(beta), mp.mpf(tau), mp.mpf(xi)
        a2 = G * G + b * b
        total = mp.mpf(0)
        big = mp.mpf(0)
        j = 0
        while True:
            sj = mp.sqrt(mp.pi / (2 * xi)) * mp.besselj(j + mp.mpf(1) / 2, xi)
            lj = mp.sqrt(mp.pi) / mp.factorial(j) * (tau / (2 * b)) ** (j + mp.mpf(1) / 2) * \
                mp.besselj(j + mp.mpf(1) / 2, b * tau)
            term = xi ** (j + 1) * sj / (2 ** j * mp.factorial(j)) * a2 ** j * lj
            total += term
            big = max(big, abs(term))
            if j > 4 and abs(term) < tol * max(big, mp.mpf(1e-300)) and j > xi and j > b * tau:
                break
            j += 1
            if j > 4000:
                raise RuntimeError("impulse series did not converge")
        return float(total)


def svea_series(a, tau, xi, dps=50):
    """Exact impulse response of the envelope equation d_tau^2 d_xi n = a n + delta(xi)
    delta(tau) (Sec. III.B after the envelope approximation): Laplace-transforming in tau and
    xi gives 1/(s^2 p - a), whose inverse is n = sum_j (a xi)^j tau^(2j+1) / (j! (2j+1)!)
    (n = tau at the front).  Summed in mpmath: for imaginary a the terms rotate in phase and
    cancel to many digits."""
    with mp.workdps(dps):
        z = mp.mpc(a) * mp.mpf(xi) * mp.mpf(tau) ** 2
        term = mp.mpc(tau)
        total = mp.mpc(0)
        j = 0
        while True:
            total += term
            j += 1
            term = term * z / (j * (2 * j) * (2 * j + 1))
            if j > 8 and abs(term) < mp.mpf(10) ** (-dps + 5) * abs(total):
                break
            if j > 200000:
                raise RuntimeError("series did not converge")
        return complex(total)


def charge_impulse_series(tau, xi, G, beta, dps=40, tol=1e-30):
    """Exact response of one Fourier mode of Eq. full_master_eq to an initial charge impulse
    rho(xi, 0) = delta(xi) with no initial current (Sec. II; at k = 0 the longitudinal master
    equation of Sec. IV.A, whose envelope obeys Eq. TSI_QSA).  The Laplace transform in tau
    is s times that of impulse_series_long (a charge present at tau = 0 instead of created
    there), so n is the tau-derivative of that series, taken term by term with
    d/dtau [tau^nu J_nu(b tau)] = b tau^nu J_(nu-1)(b tau):
        n = sum_j xi^(j+1) j_j(xi)/(2^j j!) (G^2+beta^2)^j sqrt(pi)/j! b (2b)^-(j+1/2)
            tau^(j+1/2) J_(j-1/2)(b tau).
    At tau = 0 it reduces to the free plasma response sin(xi)."""
    if xi <= 0:
        return 0.0
    if beta <= 0:
        raise ValueError("beta must be positive")
    with mp.workdps(dps):
        G, b, tau, xi = mp.mpf(G), mp.mpf(beta), mp.mpf(tau), mp.mpf(xi)
        a2 = G * G + b * b
        half = mp.mpf(1) / 2
        total = mp.mpf(0)
        big = mp.mpf(0)
        j = 0
        while True:
            sj = mp.sqrt(mp.pi / (2 * xi)) * mp.besselj(j + half, xi)
            dl = mp.sqrt(mp.pi) / mp.factorial(j) * b * (2 * b) ** (-(j + half)) * tau ** (j + half) * \
                mp.besselj(j - half, b * tau)
            term = xi ** (j + 1) * sj / (2 ** j * mp.factorial(j)) * a2 ** j * dl
            total += term
            big = max(big, abs(term))
            if j > 4 and abs(term) < tol * max(big, mp.mpf(1e-300)) and j > xi and j > b * tau:
                break
            j += 1
            if j > 4000:
                raise RuntimeError("series did not converge")
        return float(total)


def asym_rear_saddle(tau, xi, G):
    """Rear asymptote with the exponent taken to the order Appendix B carries in its saddle
    value: tau h_+(alpha_s5^+) = i G tau (C - (3/2) e^(i pi/3) C^(1/3) + e^(-i pi/3)/(8 C^(1/3))),
    C = xi/(G tau).  The third term, (sqrt(3) + i)/16 (G tau)^(4/3) xi^(-1/3) in the exponent,
    is dropped in Eqs. OTSI_ST / np_large_C; it is not small unless (G tau)^4 << xi, and
    restoring it brings the asymptote onto the exact response at C >> C_cr.  Prefactor as in
    Eq. np_large_C; returns the real value 2 Re{...}."""
    C = xi / (G * tau)
    pref = 1.0 / (4 * G) * math.sqrt(2.0 / (3 * math.pi * xi))
    corr = 1 + 1.0 / (6 * C ** (2.0 / 3.0)) * complex(0.25, math.sqrt(3) / 2)
    ph = 1j * xi + 0.75 * complex(math.sqrt(3), -1) * (G * tau) ** (2.0 / 3.0) * xi ** (1.0 / 3.0) \
        + complex(math.sqrt(3), 1) / 16.0 * (G * tau) ** (4.0 / 3.0) * xi ** (-1.0 / 3.0) - 1j * math.pi / 4
    return pref * 2 * (corr * np.exp(ph)).real


def tsi_envelope_series(beta, xi, tau, dps=60):
    """Envelope equation of Sec. IV.A (Eq. TSI_QSA, d_tau^2 d_xi n = a n with
    a = (8i/3^(3/2)) Gamma_TSI^3 = i beta^2/2) for a charge present at tau = 0: the e^(-i xi)
    part of the full response at s >> beta gives n = sum_j (a xi)^j tau^(2j)/(j! (2j)!).
    Returns ln|n| (summed in mpmath; the terms rotate in phase and cancel to many digits)."""
    with mp.workdps(dps):
        w = mp.mpc(0, 1) * mp.mpf(beta) ** 2 / 2 * mp.mpf(xi) * mp.mpf(tau) ** 2
        total = mp.mpc(0)
        term = mp.mpc(1)
        j = 0
        while True:
            total += term
            j += 1
            term = term * w / (j * (2 * j) * (2 * j - 1))
            if j > 8 and abs(term) < mp.mpf(10) ** (-dps + 5) * abs(total):
                break
            if j > 200000:
                raise RuntimeError("series did not converge")
        return float(mp.log(abs(total)))
