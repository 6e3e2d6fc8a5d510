"""Pins of the oracle's stationary front (Sec. III.D: the plasma ahead of the beam held at its
tau = 0 value, F_perp(xi = 0, tau) = F_perp(xi = 0, 0)).

With a uniform disturbance S and the front held at n_p = S, d_xi n_p = 0, the model without
the gamma^-2 term is exactly Appendix C's initial-boundary problem for Eq. CFI_st_master,
Eq. extended_BC: delta n_p(tau = 0, xi) = delta n_p(tau, xi = 0) = S, d_tau delta n_p = 0 at
tau = 0.  Its solution is a double power series: with g_0 = 1 and g_k the causal response of
the plasma oscillator to g_(k-1) (g_k'' + g_k = g_(k-1), g_k(0) = g_k'(0) = 0),
    n_p = S sum_k (Gamma tau)^(2k)/(2k)! g_k(xi),
    rho = (d_xi^2 + 1) n_p = S [1 + sum_(k>=1) (Gamma tau)^(2k)/(2k)! g_(k-1)(xi)],
since d_tau^2 rho = Gamma^2 n_p term by term.  The g_k are summed here as Taylor series in xi
in 60-digit arithmetic (mpmath), independently of the oracle's cell-by-cell propagator; the
oracle must converge to it at second order in the cell width.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O


def taylor_g(kmax, nmax):
    """Taylor coefficients c[k][n] of g_k(xi) = sum_n c[k][n] xi^n, k = 0..kmax."""
    c = [[mp.mpf(0)] * (nmax + 3) for _ in range(kmax + 1)]
    c[0][0] = mp.mpf(1)
    for k in range(1, kmax + 1):
        a, b = c[k - 1], c[k]
        # (n+2)(n+1) b[n+2] + b[n] = a[n], b[0] = b[1] = 0
        for n in range(nmax + 1):
            b[n + 2] = (a[n] - b[n]) / ((n + 1) * (n + 2))
    return c


def series_rho(S, G, tau, xis, kmax=40, nmax=260):
    with mp.workdps(60):
        c = taylor_g(kmax, nmax)
        out = []
        for xi in xis:
            x = mp.mpf(xi)
            g = [mp.fsum(ck[n] * x ** n for n in range(len(ck))) for ck in c]
            gt = mp.mpf(G) * mp.mpf(tau)
            r = 1 + mp.fsum(gt ** (2 * k) / mp.factorial(2 * k) * g[k - 1] for k in range(1, kmax + 1))
            out.append(float(S * r))
        return np.array(out)


def test_taylor_g_against_closed_forms():
    """g_1 = 1 - cos xi and g_2 = 1 - cos xi - (xi/2) sin xi solve the recursion."""
    with mp.workdps(40):
        c = taylor_g(2, 120)
        for x in (0.3, 2.0, 7.5):
            g1 = mp.fsum(c[1][n] * mp.mpf(x) ** n for n in range(len(c[1])))
            g2 = mp.fsum(c[2][n] * mp.mpf(x) ** n for n in range(len(c[2])))
            assert abs(g1 - (1 - mp.cos(x))) < 1e-25
            assert abs(g2 - (1 - mp.cos(x) - x / 2 * mp.sin(x))) < 1e-25


def _oracle_rho(N, L, n_steps, tau, S, k, nb, gamma, flags, front):
    beam = O.Beam([(-1.0, 1.0, nb)], gamma, N, L / N, flags=flags)
    st = O.seed(beam, [k], O.SEED_UNIFORM, S)
    O.run(beam, [k], tau / n_steps, n_steps, st, want_fields=False, want_max=False, front=front)
    return -st.n[0, 0, :]        # rho = q n with q = -1


def test_stationary_front_is_appendix_c_problem():
    nb, gamma, k, S, L = 0.01, 1000.0, 2.0, 1e-6, 20.0
    G = math.sqrt(nb / gamma) * k / math.sqrt(1 + k * k)
    tau = 3.0 / G
    flags = O.DROP_LONGITUDINAL | O.STATIONARY_FRONT
    errs = []
    for N in (400, 800):
        rho = _oracle_rho(N, L, 200, tau, S, k, nb, gamma, flags, front=S)
        h = L / N
        cells = [int(x / h) for x in (0.6, 3.1, 9.7, 19.4)]
        ref = series_rho(S, G, tau, [(j + 0.5) * h for j in cells])
        got = rho[cells]
        assert np.max(np.abs(got.imag)) < 1e-20
        errs.append(np.max(np.abs(got.real - ref) / np.abs(ref)))
    # second order in the cell width, and close at the finer grid
    assert errs[1] < 5e-5
    assert 3.0 < errs[0] / errs[1] < 5.0
    # the causal front (n_p = 0 ahead of the beam) is a different problem: far off the series
    rho_c = _oracle_rho(800, L, 200, tau, S, k, nb, gamma, O.DROP_LONGITUDINAL, front=None)
    h = L / 800
    ref = series_rho(S, G, tau, [0.6 // h * h + 0.5 * h])
    assert abs(rho_c[int(0.6 / h)].real - ref[0]) / abs(ref[0]) > 1e-2


def test_stationary_front_needs_values_and_scales_with_them():
    """Linearity in the front value: F = 0 is the causal front; the response to (S, F) is the
    sum of the responses to (S, 0) and (0, F) (an exact property of the linear model)."""
    nb, gamma, k, S, L, N = 0.01, 1000.0, 1.3, 1e-6, 10.0, 200
    beam = O.Beam([(-1.0, 1.0, nb)], gamma, N, L / N, flags=O.STATIONARY_FRONT)
    st = O.seed(beam, [k], O.SEED_UNIFORM, S)
    with pytest.raises(ValueError):
        O.run(beam, [k], 10.0, 2, st.copy(), want_fields=False, want_max=False)
    G = math.sqrt(nb / gamma) * k / math.sqrt(1 + k * k)
    dt = 0.02 / G
    a = st.copy()
    O.run(beam, [k], dt, 50, a, want_fields=False, want_max=False, front=(2 + 1j) * S)
    b = st.copy()
    O.run(beam, [k], dt, 50, b, want_fields=False, want_max=False, front=0.0)
    z = O.ModeState.zeros(1, beam)
    O.run(beam, [k], dt, 50, z, want_fields=False, want_max=False, front=(2 + 1j) * S)
    causal = O.Beam([(-1.0, 1.0, nb)], gamma, N, L / N)
    c = st.copy()
    O.run(causal, [k], dt, 50, c, want_fields=False, want_max=False)
    assert np.array_equal(b.n, c.n) and np.array_equal(b.pz, c.pz) and np.array_equal(b.pt, c.pt)
    scale = np.max(np.abs(a.n))
    assert np.max(np.abs(a.n - (b.n + z.n))) < 1e-13 * scale
    assert np.max(np.abs(z.n)) > 1e-3 * scale
    # renormalization divides the state by powers of two: the front value follows it
    r = st.copy()
    O.run(beam, [k], dt, 50, r, renorm=True, want_fields=False, want_max=False, front=(2 + 1j) * S)
    assert r.log2_scale[0] != 0
    assert np.max(np.abs(r.n * 2.0 ** r.log2_scale[0] - a.n)) < 1e-13 * scale
