"""Pins of the growth-map definitions (oracle/growth.py): closed forms of the Hann-weighted
window (constant fields, the weight sum, a sinusoidal modulation, brute force), the model's own
fields at tau = 0 against the baseline's first term, the baseline's joins and limits, the query coordinates (box corners, the
inverse map of the network inputs), the bin order and the plain per-bin 99th percentile."""
import math

import mpmath as mp
import numpy as np

from oracle import growth as Gr


def test_window_cells():
    assert Gr.window_cells(0.1) == 126          # 4 pi / 0.1 = 125.66
    assert Gr.window_cells(100.0) == 1
    assert Gr.window_cells(4 * math.pi / 10.4) == 10


def test_hann_weight_sum_full_window():
    """sum_{i<W} sin^2(pi (i+1/2)/W) = W/2 exactly for W >= 2 (the cosines of W >= 2 equally
    spaced angles sum to zero); one cell has the single weight 1."""
    assert Gr.hann_weights(1)[0] == 1.0
    for W in (2, 7, 126, 515):
        assert abs(math.fsum(Gr.hann_weights(W)) - W / 2) < 1e-12 * W


def test_constant_field_growth_is_log_amplitude():
    # |E| = |B| = a S on every cell: A^2/S^2 = 2 a^2, G = ln a + ln(2)/2 everywhere
    a, S = 37.0, 1e-6
    le = np.full(300, math.log(a * S))
    G = Gr.windowed_growth(le, le, 0.1, S)
    assert np.max(np.abs(G - (math.log(a) + 0.5 * math.log(2)))) < 1e-13


def test_sinusoidal_modulation_closed_form():
    """A^2 = 1 + cos(theta (j + 1/2) + phi) on the cells (|B| = 0): for a full window the
    weighted sum is W/2 + Re(e^{i(theta (j+1/2) + phi)} sum_i w_i e^{-i theta i}), with
    sum_i w_i e^{-i theta i} = (1/2) sum e^{-i theta i} - (1/4) sum (e^{i pi/W} e^{i(2pi/W - theta) i}
    + e^{-i pi/W} e^{-i(2 pi/W + theta) i}), three geometric series summed in mpmath."""
    h = 0.05
    W = Gr.window_cells(h)
    theta, phi = 2.0 * h, 0.3            # the A^2 ripple of a plasma oscillation: period pi
    n = 3 * W
    a2 = 1.0 + np.cos(theta * (np.arange(n) + 0.5) + phi)
    le = 0.5 * np.log(a2)
    G = Gr.windowed_growth(le, np.full(n, -np.inf), h, 1.0)

    def geo(z, m):
        return (1 - z ** m) / (1 - z)
    with mp.workdps(40):
        Wm = mp.mpf(W)
        s = geo(mp.expj(-theta), W) / 2 - (mp.expj(mp.pi / Wm) * geo(mp.expj(2 * mp.pi / Wm - theta), W) +
                                         mp.expj(-mp.pi / Wm) * geo(mp.expj(-2 * mp.pi / Wm - theta), W)) / 4
        for j in (W - 1, W + 17, 2 * W + 5):
            ref = 0.5 * mp.log((Wm / 2 + mp.re(mp.expj(theta * (j + 0.5) + phi) * s)) / (Wm / 2))
            assert abs(G[j] - float(ref)) < 1e-12
    # the ripple left at this cell width: under 1e-3 in G, against 2e-2 for a box of one wavelength
    assert np.ptp(G[W:]) < 2e-3


def test_brute_force_small():
    rng = np.random.default_rng(5)
    h = 4 * math.pi / 7                  # W = 7
    n = 20
    le = rng.uniform(-3, 2, n)
    lb = rng.uniform(-3, 2, n)
    G = Gr.windowed_growth(le, lb, h, 0.5)
    W = 7
    w = [math.sin(math.pi * (i + 0.5) / W) ** 2 for i in range(W)]
    for j in range(n):
        terms = [w[i] * (math.exp(2 * le[j - i]) + math.exp(2 * lb[j - i])) / 0.25 for i in range(min(j + 1, W))]
        ref = 0.5 * math.log(math.fsum(terms) / math.fsum(w[:min(j + 1, W)]))
        assert abs(G[j] - ref) < 1e-13


def test_baseline_at_tau_zero_matches_model_fields():
    """At tau = 0 the extended disturbance rho = S with the plasma at rest ahead of the front
    has n_p = S (1 - cos xi), so E_par = -kappa S sin xi, E_perp = -i k kappa S cos xi and
    B_perp = -i k kappa S (R3 fields): the window average of A^2/S^2 far from the front is
    kappa^2 (1/2 + k^2/2 + k^2), the baseline's first term (1e-4 at this cell width)."""
    h = 200.0 / 8192
    x = (np.arange(2000) + 0.5) * h
    for k in (0.05, 0.7, 4.0):
        kap = 1.0 / (1.0 + k * k)
        le = 0.5 * np.log(kap ** 2 * (np.sin(x) ** 2 + k * k * np.cos(x) ** 2))
        lb = np.full(len(x), math.log(k * kap))
        G = Gr.windowed_growth(le, lb, h, 1.0)
        assert abs(G[-1] - Gr.field_level(k)) < 1e-4


def test_box_corners_and_network_inputs():
    lo = np.array([[math.log(1e-3), math.log(10.0), 0.05, 0.0, 0.0]])
    hi = np.array([[math.log(1e-1), math.log(1e4), 4.0, 200.0, 10.0 * math.sqrt(1e4 / 1e-1)]])
    assert np.allclose(Gr.box_coords(lo), -1.0, atol=1e-14)
    assert np.allclose(Gr.box_coords(hi), 1.0, atol=1e-14)
    assert abs(Gr.tau_final(0.01, 1000.0) - 10.0 * math.sqrt(1e5)) < 1e-9
    x_lo, x_hi = Gr.features(lo)[0], Gr.features(hi)[0]
    assert np.allclose(x_lo[[2, 3, 4]], -1.0, atol=1e-12) and np.allclose(x_hi[[2, 3, 4]], 1.0, atol=1e-12)
    assert abs(x_lo[1] - (math.log10(0.5) - 2.1505) / 2.4515) < 1e-12
    # the inputs determine the query: invert them
    rng = np.random.default_rng(2)
    n = 50
    nb, g = 10 ** rng.uniform(-3, -1, n), 10 ** rng.uniform(1, 4, n)
    q = np.stack([np.log(nb), np.log(g), rng.uniform(0.05, 4, n), rng.uniform(0, 200, n),
                  rng.uniform(0, 1, n) * 10 * np.sqrt(g / nb)], 1)
    x = Gr.features(q)
    nb2 = 10 ** (x[:, 0] - 2)
    k2 = 0.05 * 80 ** ((x[:, 2] + 1) / 2)
    g2 = 10 ** (x[:, 1] * 2.4515 + 2.1505) / k2
    xi2 = 200 * ((x[:, 3] + 1) / 2) ** 2
    t2 = Gr.T_MAX * ((x[:, 4] + 1) / 2) ** 2
    tau2 = t2 / (np.sqrt(nb2 / g2) * k2 / np.sqrt(1 + k2 * k2))
    assert np.allclose(np.stack([np.log(nb2), np.log(g2), k2, xi2, tau2], 1), q, rtol=1e-10, atol=1e-9)


def test_baseline_joins():
    """J(a, b) = ln(e^a + e^b - 1) and M(a, b) = -ln(e^-a + e^-b - e^-(a+b)) on a, b >= 0:
    symmetric, 0 at the origin, J(a, 0) = a, M(a, 0) = 0, max <= J <= max + ln 2,
    min - ln 2 <= M <= min, and both within 2 e^-|a-b| of max and min once the smaller
    argument exceeds 3."""
    J, M = Gr.join_up, Gr.join_down
    rng = np.random.default_rng(4)
    a, b = rng.uniform(0, 30, 2000), rng.uniform(0, 30, 2000)
    assert np.allclose(J(a, b), J(b, a), rtol=0, atol=1e-12) and np.allclose(M(a, b), M(b, a), rtol=0, atol=1e-12)
    assert J(0.0, 0.0) == 0.0 and M(0.0, 0.0) == 0.0
    assert np.allclose(J(a, 0.0), a, rtol=0, atol=1e-12) and np.allclose(M(a, 0.0), 0.0, rtol=0, atol=1e-12)
    hi, lo = np.maximum(a, b), np.minimum(a, b)
    assert np.all(J(a, b) >= hi - 1e-12) and np.all(J(a, b) <= hi + math.log(2) + 1e-12)
    assert np.all(M(a, b) <= lo + 1e-12) and np.all(M(a, b) >= lo - math.log(2) - 1e-12)
    big = lo > 3.0
    d = np.abs(a - b)[big]
    assert np.all(J(a, b)[big] - hi[big] <= 2 * np.exp(-d) + 1e-12)
    assert np.all(lo[big] - M(a, b)[big] <= 2 * np.exp(-d) + 1e-12)


def test_baseline_growth_terms_against_the_exponents():
    """The two spatiotemporal terms against the exponents of the paper: F - (2 sqrt(t xi) - 2)
    (Eq. CFI_ST) lies in (0, 1/sqrt(t xi)], O - ((3 sqrt(3)/4) t_e^(2/3) xi^(1/3) - 3)
    (Eq. OTSI_ST) in (0, z^(-2/3)]; both start as the first terms of their series, t xi and
    z = (3 sqrt(3)/64) t_e^2 xi."""
    rng = np.random.default_rng(6)
    t, xi = rng.uniform(0.5, 20, 500), rng.uniform(1, 200, 500)
    y = t * xi
    d = Gr.front_growth(t, xi) - (2 * np.sqrt(y) - 2)
    assert np.all(d > 0) and np.all(d <= 1 / np.sqrt(y))
    z = 3 * math.sqrt(3) / 64 * t * t * xi
    d = Gr.otsi_growth(t, xi) - (3 * math.sqrt(3) / 4 * t ** (2 / 3) * xi ** (1 / 3) - 3)
    assert np.all(d > 0) and np.all(d <= z ** (-2 / 3))
    assert abs(Gr.front_growth(1e-4, 1.0) / 1e-4 - 1) < 1e-4
    assert abs(Gr.otsi_growth(1e-3, 64 / (3 * math.sqrt(3))) / 1e-6 - 1) < 1e-5


def test_baseline_limits():
    """The assembled baseline: the field level at tau = 0 at every xi; at small t the OTSI
    series' first term, B - level = (3 sqrt(3)/64) t_e^2 xi to first order, with
    t_e^2 = t^2 (1 + 1/(gamma k)^2); deep in the beam (xi >> t) the OTSI term, at
    gamma k = 1/2 with its rate raised by sqrt 5; at the front the sum of the two terms'
    slopes in xi, below the temporal growth ln cosh t."""
    nb, g, k = 0.01, 1000.0, 2.0
    lev = float(Gr.field_level(k))

    def B(t, xi, gam=g, kk=k):
        Gk = math.sqrt(nb / gam) * kk / math.sqrt(1 + kk * kk)
        return float(Gr.baseline(np.array([[math.log(nb), math.log(gam), kk, xi, t / Gk]]))[0])
    for xi in (0.0, 0.3, 30.0, 200.0):
        assert abs(B(0.0, xi) - lev) < 1e-14
    te2 = 1 + 1 / (g * k) ** 2
    for t, xi in ((1e-3, 100.0), (2e-4, 20.0)):
        z = 3 * math.sqrt(3) / 64 * t * t * te2 * xi
        assert abs((B(t, xi) - lev) / z - 1) < 2e-2
    t, xi = 8.0, 150.0
    assert abs(B(t, xi) - lev - float(Gr.otsi_growth(t * math.sqrt(te2), xi))) < 1e-6
    k5 = 0.05
    assert abs(B(t, xi, gam=10.0, kk=k5) - float(Gr.field_level(k5)) -
               float(Gr.otsi_growth(t * math.sqrt(5.0), xi))) < 1e-6
    # at the front both spatiotemporal terms start linearly in xi and add:
    # (B - level)/xi -> t + (3 sqrt(3)/64) t_e^2 once ln cosh t >> 1
    t, xi = 9.0, 1e-5
    assert abs((B(t, xi) - lev) / xi / (t + 3 * math.sqrt(3) / 64 * t * t * te2) - 1) < 1e-3
    assert B(t, 0.3) - lev < math.log(math.cosh(t))


def test_bin_order():
    x = np.array([[-1, -1, -1, -1, -1], [1, 1, 1, 1, 1], [-1, -1, -1, -1, -0.74], [-0.74, -1, -1, -1, -1]], float)
    assert list(Gr.bin_of(x)) == [0, 8 ** 5 - 1, 1, 8 ** 4]


def test_p99_table_definition():
    # 100 errors 1e-3 .. 0.1 in one bin: the 99th smallest is 0.099
    b = np.zeros((100, 5))
    err = np.arange(1, 101) * 1e-3
    t = Gr.p99_table(b, err)
    assert abs(t[int(Gr.bin_of(b[:1])[0])] - 0.099) < 1e-15
    assert np.sum(t >= 0) == 1
    # 250 errors: the 248th smallest
    err = np.random.default_rng(1).permutation(np.arange(250.0))
    assert Gr.p99_table(np.zeros((250, 5)), err)[int(Gr.bin_of(b[:1])[0])] == 247.0
    # fewer than 32 examples: no estimate
    assert np.all(Gr.p99_table(b[:31], err[:31]) == -1)
