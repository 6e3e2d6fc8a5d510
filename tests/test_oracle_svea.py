"""Pins of the envelope-approximation (SVEA) oracle, oracle/svea.py (CPU only): the exact
impulse response of the envelope equation of Sec. III.B, the growth exponent the paper
quotes for it, the coefficient against Eq. CFI_temporal, and trivial and linear cases."""
import math

import numpy as np
import pytest

from exact_refs import gamma_cfi, svea_series
from oracle import svea as S

E = (-1.0, 1.0)
P = (1.0, 1.0)


def test_converges_to_exact_impulse_response():
    """Second order in the cell size (and fourth in tau) towards
    sum_j (a xi)^j tau^(2j+1) / (j! (2j+1)!) with a = i G^2 / 2."""
    G = 0.02
    a = np.array([0.5j * G * G])
    tau, L = 200.0, 8.0
    errs = []
    for N, dt in ((64, 5.0), (128, 2.5), (256, 1.25)):
        h = L / N
        _, n, m = S.run(a, N, h, dt, int(round(tau / dt)), out_every=10 ** 9)
        xi = (np.arange(N) + 0.5) * h
        ref = np.array([svea_series(a[0], tau, x) for x in xi])
        errs.append(np.max(np.abs(n[:, 0] - ref)) / np.max(np.abs(ref)))
    assert errs[-1] < 2e-5
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_paper_growth_exponent():
    """Sec. III.B: the envelope grows as exp((3 sqrt(3)/4) (G tau)^(2/3) xi^(1/3)).  Between
    two late times the exact response's log grows by that exponent's increment (a wrong
    coefficient, e.g. i G^2 for i G^2 / 2, would change it by 2^(1/3))."""
    G = 0.02
    a = 0.5j * G * G
    for xi in (20.0, 50.0):
        t1, t2 = 2000.0, 4000.0
        d = math.log(abs(svea_series(a, t2, xi))) - math.log(abs(svea_series(a, t1, xi)))
        p = S.envelope_exponent(G, t2, xi) - S.envelope_exponent(G, t1, xi)
        assert abs(d / p - 1.0) < 0.01


@pytest.mark.parametrize("species,gamma,k", [([E + (0.01,)], 1000.0, 2.0), ([E + (0.02,), P + (0.02,)], 2e4, 3.0)])
def test_coefficient_is_half_i_gamma_cfi_squared(species, gamma, k):
    a = S.svea_coefficient(species, gamma, [k])[0]
    assert a.real == 0.0
    assert abs(a.imag / (0.5 * gamma_cfi(species, gamma, k) ** 2) - 1.0) < 1e-14


def test_zero_coefficient_is_linear_in_tau():
    """a = 0: d_tau m = 0, so m stays 1 and n = tau in every cell (RK4 exact here)."""
    sn, n, m = S.run(np.array([0j, 0j]), 16, 0.5, 0.75, 8)
    assert np.max(np.abs(m - 1.0)) == 0.0
    assert np.max(np.abs(n - 6.0)) <= 1e-14


def test_linearity_power_of_two():
    a = np.array([0.5j * 0.03 ** 2, 0.5j * 0.01 ** 2])
    n0, m0 = S.impulse_state(2, 32)
    _, n1, m1 = S.run(a, 32, 0.25, 10.0, 12, n=n0.copy(), m=m0.copy())
    _, n2, m2 = S.run(a, 32, 0.25, 10.0, 12, n=8.0 * n0, m=8.0 * m0)
    assert np.array_equal(n2, 8.0 * n1) and np.array_equal(m2, 8.0 * m1)
