"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage of the paper it relies on.  A plausible mistake in the oracle
(a dropped term, a wrong sign or index, a wrong coefficient) fails at least one of them:
  - the plasma march against its Green's function (both operators),
  - temporal CFI against the discrete RK4 closed form and Eq. CFI_temporal (coefficients,
    species sum, q^2/m, gamma^-1, kappa),
  - the impulse response against the exact series of Eq. n_alpha_xi and Appendix A's Bessel
    form (transverse coupling, causality, the front condition),
  - the longitudinal term against the exact impulse response with beta != 0,
  - the Fig.-3 printed growth rate,
  - zero density, linearity, species collapse, convergence orders.
"""
import json
import math
import os

import numpy as np
import pytest

from helpers import windowed_log_ratio
from exact_refs import (asym_critical, asym_front, front_limit_exact, gamma_cfi,
                        impulse_series, impulse_series_long, rk4_growth_factor, xi_transition)

GOLD = os.path.join(os.path.dirname(__file__), "golden")
E = (-1.0, 1.0)
P = (1.0, 1.0)


def load_golden(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------------------- generator
def test_splitmix64_published_vectors(oracle):
    g = load_golden("splitmix64_seed0.json")
    got = [oracle.splitmix64(0, i) for i in range(len(g["outputs_hex"]))]
    assert got == [int(h, 16) for h in g["outputs_hex"]]


def test_u53_range_and_uniformity(oracle):
    u = np.array([oracle.u53(oracle.splitmix64(7, i)) for i in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    # Kolmogorov-Smirnov distance of 20000 uniform draws: 1.95/sqrt(n) is the 0.1% level
    s = np.sort(u)
    d = np.max(np.maximum(np.arange(1, len(s) + 1) / len(s) - s, s - np.arange(len(s)) / len(s)))
    assert d < 1.95 / math.sqrt(len(s))


# ------------------------------------------------------------------------- plasma march
def _green_restoring(rho, h, x):
    """n(x) = int_0^x sin(x - s) rho(s) ds and its derivative for cell-constant rho."""
    n = 0.0 + 0.0j
    d = 0.0 + 0.0j
    for j, r in enumerate(rho):
        a, b = j * h, min((j + 1) * h, x)
        if a >= x:
            break
        n += r * (math.cos(x - b) - math.cos(x - a))
        d += r * (-math.sin(x - b) + math.sin(x - a))
    return n, d


def _green_free(rho, h, x):
    """n(x) = int_0^x (x - s) rho(s) ds (operator d_xi^2 alone)."""
    n = 0.0 + 0.0j
    d = 0.0 + 0.0j
    for j, r in enumerate(rho):
        a, b = j * h, min((j + 1) * h, x)
        if a >= x:
            break
        n += r * ((x - a) ** 2 - (x - b) ** 2) / 2.0
        d += r * (b - a)
    return n, d


@pytest.mark.parametrize("restoring", [True, False])
def test_march_equals_green_function(oracle, restoring):
    """Eq. plasma_oscillations_QSA with n_p = d_xi n_p = 0 ahead of the front: the march must
    equal the causal Green's-function convolution for a cell-constant source."""
    rng = np.random.default_rng(1)
    N, h = 40, 0.37
    rho = rng.normal(size=N) + 1j * rng.normal(size=N)
    beam = oracle.Beam([E + (0.01,)], 100.0, N, h, flags=0 if restoring else oracle.NO_RESTORING)
    npc, dnc, dnf = oracle.march(beam, rho)
    green = _green_restoring if restoring else _green_free
    for j in range(N):
        n, d = green(rho, h, (j + 0.5) * h)
        assert abs(npc[j] - n) < 1e-11 * (1 + abs(n))
        assert abs(dnc[j] - d) < 1e-11 * (1 + abs(d))
        n, d = green(rho, h, (j + 1) * h)
        assert abs(dnf[j] - d) < 1e-11 * (1 + abs(d))


# ------------------------------------------------------------------------- temporal CFI
@pytest.mark.parametrize("species,gamma,k,flags", [
    ([E + (0.01,)], 1000.0, 2.0, 0),
    ([E + (0.03,), P + (0.03,)], 2000.0, 5.0, 0),
    ([E + (0.05,)], 30.0, 0.7, 1),
    ([(2.0, 7.0, 0.02)], 50.0, 3.0, 0),
])
def test_temporal_cfi_rk4_closed_form(oracle, species, gamma, k, flags):
    """Uniform disturbance with the plasma ahead of the front in equilibrium (Appendix C's
    extended disturbance, K = S cosh(Gamma tau)): n_p = rho everywhere, so the state obeys
    rho'' = Gamma_CFI^2 rho exactly and RK4 gives S [R(z)^n + R(-z)^n]/2, z = Gamma dtau."""
    N, h, S = 12, 0.2, 1e-6
    beam = oracle.Beam(species, gamma, N, h, flags=flags | oracle.STEADY_INFLOW)
    st = oracle.seed(beam, [k], oracle.SEED_UNIFORM, S)
    G = gamma_cfi(species, gamma, k)
    dtau, n = 0.3 / G, 40
    oracle.run(beam, [k], dtau, n, st, want_fields=False, want_max=False)
    rho, jpar, jperp = oracle.collapse(beam, st)
    ref = S * (rk4_growth_factor(G * dtau) ** n + rk4_growth_factor(-G * dtau) ** n) / 2
    assert np.max(np.abs(rho / ref - 1)) < 1e-12
    assert np.max(np.abs(jpar)) == 0.0


def test_temporal_cfi_converges_to_cosh(oracle):
    """Same setup, dtau -> 0: S cosh(Gamma_CFI tau) (Eq. CFI_temporal; Appendix C, K term)."""
    sp, g, k, S = [E + (0.01,)], 1000.0, 3.0, 1.0
    G = gamma_cfi(sp, g, k)
    beam = oracle.Beam(sp, g, 4, 0.1, flags=oracle.STEADY_INFLOW)
    T = 8.0 / G
    errs = []
    for n in (40, 80, 160):
        st = oracle.seed(beam, [k], oracle.SEED_UNIFORM, S)
        oracle.run(beam, [k], T / n, n, st, want_fields=False, want_max=False)
        rho = oracle.collapse(beam, st)[0]
        errs.append(abs(rho[0].real / math.cosh(G * T) - 1))
    assert errs[-1] < 1e-6
    # fourth order in dtau
    assert 14.0 < errs[0] / errs[1] < 18.0 and 14.0 < errs[1] / errs[2] < 18.0


# ------------------------------------------------------------------------- impulse response
def _impulse_run(oracle, N, L, T, dtau, G, flags):
    k = 1.0
    nb_over_gamma = 2.0 * G * G  # Gamma^2 = (nb/gamma) k^2/(1+k^2) with k = 1
    gamma = 12.5
    beam = oracle.Beam([E + (nb_over_gamma * gamma,)], gamma, N, L / N,
                       flags=flags | oracle.DROP_LONGITUDINAL)
    st = oracle.seed(beam, [k], oracle.SEED_FRONT_IMPULSE, 1.0)
    n = int(round(T / dtau))
    oracle.run(beam, [k], dtau, n, st, want_fields=False, want_max=False)
    return beam, oracle.mode_fields(beam, k, st)["np"]


def test_impulse_matches_exact_series(oracle):
    """Front impulse, gamma^-2 term dropped: n_p must converge (second order) to the exact
    impulse response of Eq. CFI_st_master (series of Eq. n_alpha_xi), evaluated at the
    impulse's centre-shifted positions xi_j - h/2."""
    G, L, T = 0.02, 8.0, 200.0
    errs = []
    for N, dt in ((128, 2.5), (256, 1.25), (512, 0.625)):
        beam, npc = _impulse_run(oracle, N, L, T, dt, G, 0)
        h = L / N
        idx = np.arange(4, N, max(1, N // 16))
        ref = np.array([impulse_series(T, (j + 0.5) * h - h / 2, G) for j in idx])
        errs.append(np.max(np.abs(npc[idx].real - ref)) / np.max(np.abs(ref)))
        assert np.max(np.abs(npc[idx].imag)) < 1e-12 * np.max(np.abs(ref))
    assert errs[-1] < 3e-5
    assert 3.5 < errs[0] / errs[1] < 4.8 and 3.5 < errs[1] / errs[2] < 4.8


def test_front_limit_matches_bessel(oracle):
    """Operator d_xi^2 instead of d_xi^2 + 1 (Eq. CFI_st_master_front): the exact impulse
    response of Appendix A, [I_0 - J_0](2 sqrt(G xi tau))/(2G)."""
    G, L, T = 0.02, 4.0, 300.0
    errs = []
    for N, dt in ((32, 6.0), (64, 3.0), (128, 1.5)):
        beam, npc = _impulse_run(oracle, N, L, T, dt, G, oracle.NO_RESTORING)
        h = L / N
        idx = np.arange(2, N, max(1, N // 16))
        ref = np.array([front_limit_exact(T, (j + 0.5) * h - h / 2, G) for j in idx])
        errs.append(np.max(np.abs(npc[idx].real - ref) / np.abs(ref)))
    assert errs[-1] < 1e-3
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7


def test_exact_series_against_paper_asymptotes():
    """The exact series itself, against the paper's leading asymptotes at its Fig.-9 setting
    Gamma = 0.02 (Appendix B: Eqs. np_small_C, np_C_cr), improving with tau as the paper
    reports; and its xi -> 0 limit, Appendix A's Bessel form."""
    G = 0.02
    e200 = impulse_series(200, 0.004 * 200, G) / asym_front(200, 0.004 * 200, G) - 1
    e400 = impulse_series(400, 0.004 * 400, G) / asym_front(400, 0.004 * 400, G) - 1
    assert abs(e400) < 0.05 and abs(e400) < abs(e200)
    c200 = impulse_series(200, xi_transition(G, 200), G) / asym_critical(200, G) - 1
    c400 = impulse_series(400, xi_transition(G, 400), G) / asym_critical(400, G) - 1
    assert abs(c400) < 0.07 and abs(c400) < abs(c200)
    assert abs(impulse_series(300, 0.01, G) / front_limit_exact(300, 0.01, G) - 1) < 1e-4


# ------------------------------------------------------------------------- invariances
def test_zero_density_freezes_state(oracle):
    """Omega = 0 (n_b = 0): in Eq. beam_continuity every density rate carries a factor n0, so
    the densities, and with them the plasma response and the fields, stay bitwise fixed;
    the beam currents n0 v stay zero (test-particle velocities may still respond)."""
    beam = oracle.Beam([E + (0.0,)], 1000.0, 32, 0.1)
    st = oracle.seed(beam, [0.5, 2.0], oracle.SEED_NOISE, 1e-6, rng_seed=3)
    st0 = st.copy()
    ln_e, ln_b, mx = oracle.run(beam, [0.5, 2.0], 10.0, 5, st)
    assert np.array_equal(st.n, st0.n)
    assert np.all(mx == mx[0])
    for m in range(2):
        rho, jpar, jperp = oracle.collapse(beam, st, m)
        assert np.max(np.abs(jpar)) == 0.0 and np.max(np.abs(jperp)) == 0.0


def test_linearity_power_of_two(oracle):
    """The model is linear: a seed scaled by 2^m gives the state scaled by 2^m bitwise and
    ln-fields shifted by m ln 2."""
    beam = oracle.Beam([E + (0.01,)], 1000.0, 64, 20.0 / 64)
    k = [0.3, 1.7, 3.9]
    a = oracle.seed(beam, k, oracle.SEED_NOISE, 1e-6, rng_seed=11)
    b = oracle.seed(beam, k, oracle.SEED_NOISE, 1e-6 * 2.0 ** 7, rng_seed=11)
    ea, _, ma = oracle.run(beam, k, 50.0, 20, a, out_every=5)
    eb, _, mb = oracle.run(beam, k, 50.0, 20, b, out_every=5)
    assert np.array_equal(b.n, a.n * 2.0 ** 7)
    assert np.allclose(eb - ea, 7 * math.log(2.0), atol=1e-12, rtol=0)
    assert np.allclose(mb - ma, 7 * math.log(2.0), atol=1e-12, rtol=0)


def test_renormalization_is_exact(oracle):
    """Power-of-two renormalization changes nothing but the stored exponent."""
    beam = oracle.Beam([E + (0.01,)], 1000.0, 48, 0.4)
    k = [0.8, 2.5]
    a = oracle.seed(beam, k, oracle.SEED_NOISE, 1e-6, rng_seed=5)
    b = a.copy()
    ea, ba, ma = oracle.run(beam, k, 60.0, 12, a, renorm=False)
    eb, bb, mb = oracle.run(beam, k, 60.0, 12, b, renorm=True)
    assert np.max(np.abs(ea - eb)) < 1e-12 and np.max(np.abs(ma - mb)) < 1e-12
    scale = 2.0 ** b.log2_scale[:, None, None]
    assert np.array_equal(b.n * scale, a.n)


def test_species_collapse(oracle):
    """Only sum_s q_s^2 n_bs/m_s enters (master equation, Eq. full_master_eq): a neutral pair
    beam of n_b/2 per species equals an electron beam of n_b, whichever species carries the
    seed; a wrong charge power or sign breaks this."""
    N, h, k = 40, 0.5, [0.6, 2.2]
    e = oracle.Beam([E + (0.02,)], 500.0, N, h)
    pr = oracle.Beam([E + (0.01,), P + (0.01,)], 500.0, N, h)
    pr_rev = oracle.Beam([P + (0.01,), E + (0.01,)], 500.0, N, h)
    outs = []
    for beam in (e, pr, pr_rev):
        st = oracle.seed(beam, k, oracle.SEED_NOISE, 1e-6, rng_seed=9)
        outs.append(oracle.run(beam, k, 40.0, 15, st, out_every=3))
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.max(np.abs(x - y)) < 1e-11


# ------------------------------------------------------------------------- convergence
def test_convergence_orders(oracle):
    """Observed orders of the discrete scheme: 2 in xi (exact cell propagator of a
    cell-centred source, staggered currents) and 4 in tau (RK4)."""
    sp, g, k, L, T = [E + (0.01,)], 100.0, [1.5], 4.0, 600.0

    def final_np(N, n_t):
        beam = oracle.Beam(sp, g, N, L / N)
        st = oracle.seed(beam, k, oracle.SEED_UNIFORM, 1.0)
        oracle.run(beam, k, T / n_t, n_t, st, want_fields=False, want_max=False)
        npc = oracle.mode_fields(beam, k[0], st)["np"]
        # xi = 3.125 is a cell centre of the 16-, 48- and 144-cell grids (refinement by 3)
        j = int(round(3.125 / (L / N) - 0.5))
        assert abs((j + 0.5) * (L / N) - 3.125) < 1e-12
        return npc[j]

    # xi refinement at a fine tau step
    a, b, c = (final_np(N, 400) for N in (16, 48, 144))
    px = math.log(abs(a - b) / abs(b - c)) / math.log(3.0)
    assert 1.8 < px < 2.2
    # tau refinement at fixed xi grid
    a, b, c = (final_np(48, n) for n in (10, 20, 40))
    pt = math.log2(abs(a - b) / abs(b - c))
    assert 3.8 < pt < 4.2


# ------------------------------------------------------------------------- printed values
def test_printed_cfi_rate_fig3(oracle):
    """Sec. III.D: a pair beam of peak density 0.03 per species, gamma = 2000, k = 5 has
    Gamma_CFI ~ 5.5e-3 (printed).  Measured from the oracle's temporal growth."""
    g = load_golden("paper_printed_values.json")["fig3_peak_gamma_cfi"]
    sp, gam, k = [E + (0.03,), P + (0.03,)], 2000.0, 5.0
    beam = oracle.Beam(sp, gam, 4, 0.1, flags=oracle.STEADY_INFLOW)
    st = oracle.seed(beam, [k], oracle.SEED_UNIFORM, 1.0)
    T, n = 3000.0, 300
    oracle.run(beam, [k], T / n, n, st, want_fields=False, want_max=False)
    r1 = oracle.collapse(beam, st)[0][0].real
    oracle.run(beam, [k], T / n, n, st, want_fields=False, want_max=False)
    r2 = oracle.collapse(beam, st)[0][0].real
    rate = math.log(r2 / r1) / T
    assert abs(rate / g["value"] - 1) < g["rel_tol"]


@pytest.mark.parametrize("species,gamma,k", [
    ([E + (0.05,)], 3.0, 0.5),
    ([E + (0.02,), P + (0.02,), (2.0, 4.0, 0.01)], 2.5, 1.3),
])
def test_impulse_with_longitudinal_term(oracle, species, gamma, k):
    """Front impulse with the gamma^-2 d_xi^2 term kept (Eq. full_master_eq, one Fourier
    mode): n_p converges at second order to the exact impulse response whose Laplace form
    is sin(kappa xi)/(kappa (s^2+beta^2)), kappa^2 = (s^2-G^2)/(s^2+beta^2).  At these
    parameters the longitudinal term changes n_p by O(1), so the gamma^-3 current, the
    face-centred Omega and the flux form are all pinned."""
    w2 = sum(q * q * nb / (m * gamma) for (q, m, nb) in species)
    G = math.sqrt(w2 * k * k / (1 + k * k))
    b = math.sqrt(w2 / (gamma * gamma * (1 + k * k)))
    L, T = 8.0, 100.0
    errs = []
    for N, dt in ((128, 2.0), (256, 1.0), (512, 0.5)):
        beam = oracle.Beam(species, gamma, N, L / N)
        st = oracle.seed(beam, [k], oracle.SEED_FRONT_IMPULSE, 1.0)
        oracle.run(beam, [k], dt, int(round(T / dt)), st, want_fields=False, want_max=False)
        npc = oracle.mode_fields(beam, k, st)["np"]
        h = L / N
        idx = np.arange(4, N, max(1, N // 16))
        ref = np.array([impulse_series_long(T, (j + 0.5) * h - h / 2, G, b) for j in idx])
        ref0 = np.array([impulse_series(T, (j + 0.5) * h - h / 2, G) for j in idx])
        assert np.max(np.abs(ref0 - ref)) > 0.1 * np.max(np.abs(ref))  # the term matters here
        errs.append(np.max(np.abs(npc[idx].real - ref)) / np.max(np.abs(ref)))
    assert errs[-1] < 1.5e-4
    # second order (error components of the xi and tau discretizations may partly cancel on
    # the coarsest grid, hence the wide upper bound)
    assert 3.4 < errs[0] / errs[1] < 8.0 and 3.4 < errs[1] / errs[2] < 8.0, errs


# ------------------------------------------------------------------------- field hierarchy
@pytest.mark.parametrize("n_xi", [256, 512])
def test_field_hierarchy_behind_the_front(oracle, n_xi):
    """Sec. III.C, Fig. 2 (the 2D PIC run: pair beam, n_b = 0.02 per species, gamma = 2e4,
    k_y ~ 3): at Gamma_CFI tau = 5.63 the magnetic field dominates at xi = 2 (spatiotemporal
    CFI near the front) and the electric field at xi = 20 (spatiotemporal OTSI behind it).
    The model seeded by a front impulse reproduces both, with the field energies averaged
    over one plasma wavelength (the oscillatory OTSI response has nodes in E and B at
    different places), at two resolutions."""
    sp, gam, k = [E + (0.02,), P + (0.02,)], 2e4, 3.0
    G = gamma_cfi(sp, gam, k)
    L = 40.0
    beam = oracle.Beam(sp, gam, n_xi, L / n_xi)
    st = oracle.seed(beam, [k], oracle.SEED_FRONT_IMPULSE, 1e-6)
    tau, n = 5.63 / G, n_xi // 2
    oracle.run(beam, [k], tau / n, n, st, renorm=True, want_fields=False, want_max=False)
    f = oracle.mode_fields(beam, k, st)
    h = L / n_xi
    assert windowed_log_ratio(f["ln_e"], f["ln_b"], h, 2.0) < -0.2      # |B| dominates
    assert windowed_log_ratio(f["ln_e"], f["ln_b"], h, 20.0) > 0.4      # |E| dominates
    # the magnetic front region is about xi_tr = 2 Gamma tau / sqrt(27) long
    assert 2.0 < xi_transition(G, tau) < 2.4
