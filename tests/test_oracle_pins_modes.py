"""More pins of the FP64 oracle (CPU only): the longitudinal k = 0 mode (two-stream), the
rear spatiotemporal OTSI regime, the critical line, the transverse fields against Gauss's
law and Ampere's law, and the flux form of a xi-dependent beam profile.  Each pin has a
metric function; the last test plants one mistake at a time in a copy of the oracle
(oracle.build_variant) and checks that its pin fails.
"""
import json
import math
import os

import numpy as np
import pytest

from exact_refs import (asym_rear, asym_rear_saddle, charge_impulse_series, gamma_tsi,
                        impulse_series, tsi_envelope_series)

GOLD = os.path.join(os.path.dirname(__file__), "golden")
E = (-1.0, 1.0)
P = (1.0, 1.0)


def golden(key):
    with open(os.path.join(GOLD, "paper_printed_values.json")) as f:
        return json.load(f)[key]


def _envelope(npc, h, xi):
    """RMS of n_p over one plasma wavelength centred on xi (the envelope of a response
    oscillating at the plasma wavelength)."""
    x = (np.arange(len(npc)) + 0.5) * h
    m = np.abs(x - xi) <= math.pi
    return math.sqrt(float(np.mean(np.abs(npc[m]) ** 2)))


# ------------------------------------------------------------------ k = 0: two-stream mode
K0_BEAM = dict(nb=0.1, gamma=10.0)  # beta = sqrt(n_b / gamma^3) = 0.01


def k0_charge_impulse_error(oracle, N, dt, L=8.0, T=300.0):
    """A charge impulse rho = 1/h in cell 0 at tau = 0, no current, k = 0: relative max error
    of n_p at the cell centres against the exact response (charge_impulse_series) at the
    impulse-centred positions xi_j - h/2."""
    nb, g = K0_BEAM["nb"], K0_BEAM["gamma"]
    beta = math.sqrt(nb / g ** 3)
    h = L / N
    beam = oracle.Beam([E + (nb,)], g, N, h)
    st = oracle.ModeState.zeros(1, beam)
    st.n[0, 0, 0] = (1.0 / h) / E[0]
    oracle.run(beam, [0.0], dt, int(round(T / dt)), st, want_fields=False, want_max=False)
    npc = oracle.mode_fields(beam, 0.0, st)["np"]
    idx = np.arange(4, N, max(1, N // 16))
    ref = np.array([charge_impulse_series(T, (j + 0.5) * h - h / 2, 0.0, beta) for j in idx])
    free = np.array([math.sin((j + 0.5) * h - h / 2) for j in idx])
    assert np.max(np.abs(ref - free)) > 0.5 * np.max(np.abs(ref))  # the beam response matters here
    assert np.max(np.abs(npc[idx].imag)) == 0.0
    return float(np.max(np.abs(npc[idx].real - ref)) / np.max(np.abs(ref)))


def test_k0_charge_impulse_matches_exact_response(oracle):
    """Sec. IV.A, k = 0: with no transverse wavenumber only the gamma^-3 longitudinal current
    couples the beam to the plasma; the master equation becomes
    [d_tau^2 (d_xi^2 + 1) + sum_s omega_bs^2/gamma^2 d_xi^2] n_p = 0.  The oracle's k = 0 mode
    converges at second order to its exact Laplace-form response."""
    errs = [k0_charge_impulse_error(oracle, N, dt) for N, dt in ((64, 4.0), (128, 2.0), (256, 1.0))]
    assert errs[-1] < 2e-4, errs
    assert 3.3 < errs[0] / errs[1] < 5.0 and 3.3 < errs[1] / errs[2] < 5.0, errs


def tsi_growth_coefficient(oracle, xi=50.0, taus=(6000.0, 8000.0)):
    """Envelope growth of the k = 0 charge-impulse response of the paper's 1D PIC beam (pair
    beam, n_b = 0.6 per species, gamma = 200; Sec. IV.A) between two times at fixed xi, in
    units of Gamma_TSI xi^(1/3) d(tau^(2/3))."""
    sp, g = [E + (0.6,), P + (0.6,)], 200.0
    L, N, dt = 60.0, 1200, 5.0
    h = L / N
    beam = oracle.Beam(sp, g, N, h)
    st = oracle.ModeState.zeros(1, beam)
    st.n[0, 0, 0] = (1.0 / h) / sp[0][0]
    lns, done = [], 0.0
    for T in taus:
        oracle.run(beam, [0.0], dt, int(round((T - done) / dt)), st, want_fields=False, want_max=False,
                   renorm=True)
        done = T
        npc = oracle.mode_fields(beam, 0.0, st)["np"]
        lns.append(math.log(_envelope(npc, h, xi)) + st.log2_scale[0] * math.log(2.0))
    Gt = gamma_tsi(sp, g)
    return (lns[1] - lns[0]) / (Gt * xi ** (1 / 3) * (taus[1] ** (2 / 3) - taus[0] ** (2 / 3)))


def test_tsi_growth_against_printed_exponent(oracle):
    """Eq. TSI_QSA_analyt_GF: the k = 0 envelope grows as exp[(3/2^(2/3)) Gamma_TSI xi^(1/3)
    tau^(2/3)].  At the paper's two-stream parameters, deep in the envelope regime
    (xi/tau = 16 beta), the oracle's growth coefficient is within the golden tolerance of the
    printed one; the envelope equation's own exact response approaches the printed
    coefficient from below as the exponent grows (within 1 % at an exponent of ~580)."""
    g = golden("tsi_exponent_coefficient")
    c = tsi_growth_coefficient(oracle)
    assert abs(c / g["value"] - 1) < g["rel_tol"], c
    beta, xi = 1e-3, 40.0
    gt = math.sqrt(3.0) / 2 ** (4.0 / 3.0) * beta ** (2.0 / 3.0)
    coef = []
    for T in (1e4, 1e6):
        d = tsi_envelope_series(beta, xi, 1.5 * T, 120) - tsi_envelope_series(beta, xi, T, 120)
        coef.append(d / (gt * xi ** (1 / 3) * ((1.5 * T) ** (2 / 3) - T ** (2 / 3))))
    assert coef[0] < coef[1] and abs(coef[1] / g["value"] - 1) < 0.01, coef


# ------------------------------------------------------------------ rear: spatiotemporal OTSI
def test_exact_series_rear_asymptote():
    """Appendix B, C >> C_cr: the exact impulse response (Eq. n_alpha_xi, summed exactly)
    against the rear asymptote.  With the exponent carried to the order of Appendix B's own
    saddle value h_+(alpha_s5^+) (asym_rear_saddle) the two agree to within 2 % of the envelope
    at C = 5 and 0.3 % at C = 20, improving with C; the printed Eq. np_large_C, which drops the
    (sqrt(3) + i)/16 (G tau)^(4/3) xi^(-1/3) exponent term, is off by a third here."""
    G, GT = 0.1, 10.0
    T = GT / G
    errs = []
    for C in (5.0, 10.0, 20.0):
        xs = C * GT + np.linspace(-math.pi, math.pi, 11)
        ex = np.array([impulse_series(T, x, G) for x in xs])
        env = np.max(np.abs(ex))
        errs.append(np.max(np.abs(ex - np.array([asym_rear_saddle(T, x, G) for x in xs]))) / env)
        printed = np.max(np.abs(ex - np.array([asym_rear(T, x, G) for x in xs]))) / env
        assert printed > 0.3
    assert errs[0] < 2.5e-2 and errs[2] < 3e-3 and errs[0] > errs[1] > errs[2], errs


def rear_otsi_growth(oracle, xis=(200.0, 400.0), GTs=(10.0, 15.0)):
    """Front impulse, gamma^-2 term dropped (Eq. CFI_st_master), G = 0.1: growth of the n_p
    envelope at fixed xi between two times, as (coefficient of (G tau)^(2/3) xi^(1/3), ratio
    to the growth of asym_rear_saddle's envelope) per xi."""
    G, k, gamma = 0.1, 1.0, 12.5
    nb = 2.0 * G * G * gamma  # G^2 = (n_b/gamma) k^2/(1+k^2) with k = 1
    L, N, dt = 420.0, 8400, 0.5
    h = L / N
    beam = oracle.Beam([E + (nb,)], gamma, N, h, flags=oracle.DROP_LONGITUDINAL)
    st = oracle.seed(beam, [k], oracle.SEED_FRONT_IMPULSE, 1.0)
    lns, done = [], 0.0
    for GT in GTs:
        T = GT / G
        oracle.run(beam, [k], dt, int(round((T - done) / dt)), st, want_fields=False, want_max=False, renorm=True)
        done = T
        npc = oracle.mode_fields(beam, k, st)["np"]
        lns.append([math.log(_envelope(npc, h, xi)) + st.log2_scale[0] * math.log(2.0) for xi in xis])
    out = []
    for i, xi in enumerate(xis):
        d = lns[1][i] - lns[0][i]
        asym = []
        for GT in GTs:
            xs = xi + np.linspace(-math.pi, math.pi, 41)
            asym.append(math.log(math.sqrt(np.mean(np.array([asym_rear_saddle(GT / G, x, G) for x in xs]) ** 2))))
        coef = d / (xi ** (1 / 3) * (GTs[1] ** (2 / 3) - GTs[0] ** (2 / 3)))
        out.append((coef, d / (asym[1] - asym[0])))
    return out


def test_oracle_rear_otsi_exponent(oracle):
    """Sec. III.B / Eq. OTSI_ST: deep behind the front (C = xi/(Gamma tau) from 13 to 40) the
    envelope of the full model's impulse response grows as exp[(3 sqrt(3)/4) (Gamma tau)^(2/3)
    xi^(1/3)] (golden coefficient, here within 4 % and closer at larger C), and within 1 % as
    the asymptote with Appendix B's next exponent term."""
    g = golden("otsi_exponent_coefficient")
    (c200, r200), (c400, r400) = rear_otsi_growth(oracle)
    assert abs(c400 / g["value"] - 1) < 0.04 and abs(c400 / g["value"] - 1) < abs(c200 / g["value"] - 1)
    assert abs(r200 - 1) < 0.01 and abs(r400 - 1) < 0.01, (r200, r400)


def test_critical_line_rate_and_transition():
    """Sec. III.B and Appendix B: the roots of z^3 + z^2 - C^2 = 0 (Eq. P_z) are all real
    exactly below C_cr = 2/sqrt(27) (golden transition coefficient); an observer moving with
    xi = C_cr Gamma tau sees the exact impulse response grow at (4/3) sqrt(2/3) Gamma (golden
    critical-line rate; Eq. np_C_cr, with its (Gamma tau)^(-1/3) prefactor)."""
    c_tr = golden("transition_coefficient")["value"]
    rate = golden("critical_line_rate")["value"]
    assert abs(c_tr - 2 / math.sqrt(27)) < 1e-12 and abs(rate - 4 / 3 * math.sqrt(2 / 3)) < 1e-12
    for C, real in ((c_tr * (1 - 1e-3), True), (c_tr * (1 + 1e-3), False)):
        r = np.roots([1.0, 1.0, 0.0, -C * C])
        assert bool(np.all(np.abs(r.imag) < 1e-9)) == real
    G = 0.02
    t1, t2 = 40.0 / G, 60.0 / G
    n1, n2 = impulse_series(t1, c_tr * G * t1, G), impulse_series(t2, c_tr * G * t2, G)
    measured = (math.log(n2 / n1) + math.log(t2 / t1) / 3.0) / (G * (t2 - t1))
    assert abs(measured / rate - 1) < 0.01, measured


# ------------------------------------------------------------------ fields: Gauss and Ampere
def field_law_errors(oracle, N, k=1.3, L=10.0):
    """A smooth charge density rho(xi) (no current): the oracle's |B_perp| and |E_perp| against
    Ampere's law (x component) and Gauss's law with the paper's v_px = Psi, using central
    differences of its own E_par:
        i k B_perp = rho - Psi + d_xi E_par,     i k E_perp = rho - n_p + d_xi E_par.
    Returns the two relative max errors over the interior cells."""
    h = L / N
    beam = oracle.Beam([E + (0.01,)], 100.0, N, h)
    x = (np.arange(N) + 0.5) * h
    rho = np.exp(-0.5 * (x - 5.0) ** 2) * (1 + 0.5j) * np.exp(0.7j * x)
    st = oracle.ModeState.zeros(1, beam)
    st.n[0, 0] = rho / E[0]
    f = oracle.mode_fields(beam, k, st)
    kap = 1.0 / (1.0 + k * k)
    ep, npc = f["e_par"], f["np"]
    dep = (ep[2:] - ep[:-2]) / (2 * h)
    r, n = rho[1:-1], npc[1:-1]
    b_law = np.abs(r - kap * n + dep) / k
    e_law = np.abs(r - n + dep) / k
    b = np.exp(f["ln_b"][1:-1])
    e_perp = np.sqrt(np.maximum(np.exp(2 * f["ln_e"][1:-1]) - np.abs(ep[1:-1]) ** 2, 0.0))
    return (float(np.max(np.abs(b - b_law)) / np.max(b_law)),
            float(np.max(np.abs(e_perp - e_law)) / np.max(e_law)))


def test_fields_satisfy_gauss_and_ampere(oracle):
    """Sec. II: Gauss's law div E = rho - n_p (printed there) and the x component of Ampere's
    law in the quasistatic ordering, with v_px = Psi (Sec. II) and E_par = -d_xi Psi, fix the
    transverse fields E_perp and B_perp of a mode; the oracle's fields satisfy both to second
    order in the cell width."""
    errs = [field_law_errors(oracle, N) for N in (100, 200, 400)]
    for i in range(2):
        e = [x[i] for x in errs]
        assert e[-1] < 3e-4 and 3.6 < e[0] / e[1] < 4.4 and 3.6 < e[1] / e[2] < 4.4, errs


# ------------------------------------------------------------------ xi-dependent profile
def profile_residual(oracle, N, dt=0.02, nb=0.2, g=2.0, k=1.2, L=12.0, xc=6.0, sig=1.5):
    """Gaussian beam profile, gamma = 2 so that the gamma^-2 terms are large: the residual of
    the mode form of Eq. full_master_eq_v2,
        (d_xi^2 + 1) d_tau^2 n_p = kappa [gamma^-1 k^2 Omega n_p - gamma^-3 d_xi(Omega d_xi n_p)],
    Omega = q^2 n0(xi)/m, evaluated on the oracle's state (d_tau^2 of rho = (d_xi^2+1) n_p by
    a second difference over steps of dt; d_xi(Omega d_xi n_p) from the march's face values
    of d_xi n_p with Omega of the profile itself).  Returned relative to the largest
    longitudinal term; second order in h and dt."""
    h = L / N
    x = (np.arange(N) + 0.5) * h
    prof = np.exp(-0.5 * ((x - xc) / sig) ** 2)
    beam = oracle.Beam([E + (nb,)], g, N, h, shape=prof)
    st = oracle.seed(beam, [k], oracle.SEED_UNIFORM, 1.0)
    oracle.run(beam, [k], 0.25, 8, st, want_fields=False, want_max=False)
    rhos = []
    for i in range(3):
        rhos.append(oracle.collapse(beam, st)[0].copy())
        if i < 2:
            oracle.run(beam, [k], dt, 1, st, want_fields=False, want_max=False)
    lhs = (rhos[2] - 2 * rhos[1] + rhos[0]) / dt ** 2
    npc, _, dnf = oracle.march(beam, rhos[1])
    kap = 1.0 / (1.0 + k * k)

    def omega(xx):
        return E[0] ** 2 * nb * np.exp(-0.5 * ((xx - xc) / sig) ** 2) / E[1]

    flux = omega((np.arange(N) + 1) * h) * dnf
    flux[-1] = 0.0                            # no beam behind the last face
    div = np.diff(np.concatenate([[0.0], flux])) / h
    longit = kap * div / g ** 3
    rhs = kap * (k * k * omega(x) * npc / g) - longit
    sl = slice(2, N - 2)
    return float(np.max(np.abs(lhs - rhs)[sl]) / np.max(np.abs(longit[sl])))


def test_profile_flux_form_master_equation(oracle):
    """Sec. III.D, Eqs. beam_second_eq_motion_v2 and full_master_eq_v2: for a xi-dependent
    profile the beam equations carry the extra gamma^-2 (d_xi ln n0) d_xi term; in flux form
    it is d_xi(Omega d_xi Psi).  The oracle's state satisfies the profile master equation with
    a residual that vanishes at second order."""
    r = [profile_residual(oracle, N) for N in (60, 120, 240)]
    assert r[-1] < 3e-4 and 3.3 < r[0] / r[1] < 4.7 and 3.3 < r[1] / r[2] < 4.7, r


# ------------------------------------------------------------------ planted mistakes
def _temporal_cfi_error(oracle):
    """Uniform disturbance, steady inflow: rho must grow as cosh(Gamma_CFI tau)."""
    sp, g, k = [E + (0.01,)], 1000.0, 3.0
    G = math.sqrt(0.01 / g * k * k / (1 + k * k))
    beam = oracle.Beam(sp, g, 4, 0.1, flags=oracle.STEADY_INFLOW)
    st = oracle.seed(beam, [k], oracle.SEED_UNIFORM, 1.0)
    T = 4.0 / G
    oracle.run(beam, [k], T / 200, 200, st, want_fields=False, want_max=False)
    return abs(oracle.collapse(beam, st)[0][0].real / math.cosh(G * T) - 1)


PLANTED = [
    ("EPERP_SIGN", lambda o: field_law_errors(o, 100)[1], 3e-3),
    ("BPERP_NP", lambda o: field_law_errors(o, 100)[0], 3e-3),
    ("NONFLUX", lambda o: profile_residual(o, 60), 3e-3),
    ("LONG_SIGN", lambda o: k0_charge_impulse_error(o, 64, 4.0), 2e-3),
    ("FACE_INDEX", lambda o: k0_charge_impulse_error(o, 64, 4.0), 2e-3),
    ("TRANS_SIGN", _temporal_cfi_error, 1e-6),
]


@pytest.mark.parametrize("plant,metric,bar", PLANTED, ids=[p[0] for p in PLANTED])
def test_planted_mistake_fails_its_pin(oracle, tmp_path, plant, metric, bar):
    """Each pin, at its coarsest resolution, passes on the oracle and fails by a wide margin
    on a copy with the planted mistake (a sign slip, an index slip, a dropped term)."""
    good = metric(oracle)
    assert good < bar, good
    path = oracle.build_variant(plant, str(tmp_path))
    with oracle.use_library(path):
        bad = metric(oracle)
    assert bad > 10 * bar, (plant, good, bad)
