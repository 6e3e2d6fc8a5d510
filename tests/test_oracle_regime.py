"""Pins of the E/B regime-diagnostic oracle, oracle/regime.py (CPU only).

The definition is pinned by closed forms (constant fields; a field growing geometrically
along xi, whose window sum is a geometric series), by brute force with exactly rounded sums
on small inputs, and by the paper's statements about the boundary it measures (Sec. III.B,
Fig. 1; Sec. III.C): the field in front of it is magnetically dominated and behind it
electrically, and in (xi, Gamma_CFI tau) the boundary is the same for every beam-plasma
parameter set and tends to xi_tr = 2 Gamma_CFI tau / sqrt(27) as Gamma_CFI tau grows.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from exact_refs import gamma_cfi, xi_transition
from oracle import regime as RG

E_SP = (-1.0, 1.0)
P_SP = (1.0, 1.0)


@pytest.mark.parametrize("w", [0, 3, 8])
def test_constant_fields(w):
    n = 40
    ln_e = np.full((n, 3), [0.5, -2.0, 7.0])
    ln_b = np.full((n, 3), [0.1, -1.0, 7.0])
    R = RG.log_ratio_map(ln_e, ln_b, w)
    assert np.all(np.isnan(R[:w])) and np.all(np.isnan(R[n - w:]))
    np.testing.assert_allclose(R[w:n - w], np.broadcast_to([0.4, -1.0, 0.0], (n - 2 * w, 3)), rtol=0, atol=1e-14)
    assert list(RG.first_e_cell(R)) == [w, -1, -1]


@pytest.mark.parametrize("s,w", [(0.3, 5), (-0.7, 12), (4.0, 40), (1e-3, 1)])
def test_geometric_field_closed_form(s, w):
    """ln|E_i| = s i + 3, |B| = 1: sum_{m=-w}^{w} e^{2 s (j + m)} = e^{2 s j} sinh((2w+1) s) / sinh(s),
    so R_j = 3 + s j + 1/2 ln( sinh((2w+1) s) / ((2w+1) sinh(s)) ) -- over a column spanning up to
    e^{2 s n} = e^{1600} (s = 4, n = 200): only a per-window reference keeps it finite."""
    n = 200
    i = np.arange(n, dtype=np.float64)
    R = RG.log_ratio_map(3.0 + s * i, np.zeros(n), w)[:, 0]
    c = float(mp.log(mp.sinh((2 * w + 1) * mp.mpf(s)) / ((2 * w + 1) * mp.sinh(mp.mpf(s)))) / 2)
    ref = 3.0 + s * i[w:n - w] + c
    np.testing.assert_allclose(R[w:n - w], ref, rtol=1e-13, atol=1e-12)


def _brute(ln_e, ln_b, w):
    n, m = ln_e.shape
    out = np.full((n, m), np.nan)
    for k in range(m):
        for j in range(w, n - w):
            se = math.fsum(math.exp(2 * ln_e[i, k]) for i in range(j - w, j + w + 1))
            sb = math.fsum(math.exp(2 * ln_b[i, k]) for i in range(j - w, j + w + 1))
            out[j, k] = 0.5 * math.log(se / sb)
    return out


@pytest.mark.parametrize("n,w", [(11, 0), (11, 2), (11, 5), (11, 6), (23, 9)])
def test_brute_force_small(n, w):
    rng = np.random.default_rng(n * 10 + w)
    ln_e = rng.normal(0.0, 3.0, (n, 4))
    ln_b = rng.normal(0.5, 3.0, (n, 4))
    R = RG.log_ratio_map(ln_e, ln_b, w)
    ref = _brute(ln_e, ln_b, w)
    assert np.array_equal(np.isnan(R), np.isnan(ref))
    np.testing.assert_allclose(R[~np.isnan(R)], ref[~np.isnan(ref)], rtol=0, atol=1e-13)
    hit = ref > 0
    want = [int(np.argmax(hit[:, k])) if hit[:, k].any() else -1 for k in range(4)]
    assert list(RG.first_e_cell(R)) == want


def test_special_values():
    n, w = 12, 2
    ln_e = np.zeros((n, 4))
    ln_b = np.zeros((n, 4))
    ln_e[:, 0] = -np.inf                 # no electric field: R = -inf
    ln_b[:, 1] = -np.inf                 # no magnetic field: R = +inf
    ln_e[:, 2] = -np.inf
    ln_b[:, 2] = -np.inf                 # neither: NaN
    ln_e[6, 3] = np.nan                  # a NaN spoils the windows that hold it
    R = RG.log_ratio_map(ln_e, ln_b, w)
    assert np.all(R[w:n - w, 0] == -np.inf) and np.all(R[w:n - w, 1] == np.inf)
    assert np.all(np.isnan(R[:, 2]))
    assert np.all(np.isnan(R[4:9, 3])) and np.all(R[w:4, 3] == 0.0) and np.all(R[9:n - w, 3] == 0.0)
    assert list(RG.first_e_cell(R)) == [-1, w, -1, -1]


def test_half_window_cells():
    assert RG.half_window_cells(1.0, 100.0 / 4096) == 40
    assert RG.half_window_cells(1.0, 0.04) == 25
    assert RG.half_window_cells(1.0, 0.1) == 10
    assert RG.half_window_cells(0.0, 0.1) == 0


def _crossing(species, gamma, k, g_tau, h=0.05, steps_per_unit=40):
    """Front-impulse run of one mode to Gamma_CFI tau = g_tau; the first electrically dominated
    cell of the +-1 skin-depth window map, in units of xi_tr, and the map itself."""
    G = gamma_cfi(species, gamma, k)
    L = max(24.0, 1.3 * g_tau)
    n_xi = int(round(L / h))
    beam = oracle.Beam(species, gamma, n_xi, h)
    st = oracle.seed(beam, [k], oracle.SEED_FRONT_IMPULSE, 1e-6)
    tau, n = g_tau / G, int(steps_per_unit * g_tau)
    oracle.run(beam, [k], tau / n, n, st, renorm=True, want_fields=False, want_max=False)
    f = oracle.mode_fields(beam, k, st)
    R = RG.log_ratio_map(f["ln_e"], f["ln_b"], RG.half_window_cells(1.0, h))
    j = int(RG.first_e_cell(R)[0])
    assert j >= 0
    return (j + 0.5) * h / xi_transition(G, tau), R[:, 0]


def test_boundary_independent_of_beam_parameters(oracle):
    """Sec. III.B: in (xi, Gamma_CFI tau) the CFI/OTSI boundary does not depend on n_b, gamma_b
    (ultrarelativistic, dilute) or k.  Three beams at Gamma_CFI tau = 12: the measured boundary
    agrees to within one cell (0.05 / xi_tr = 1.1 %)."""
    sets = [([E_SP + (0.02,), P_SP + (0.02,)], 2e4, 3.0), ([E_SP + (0.01,)], 1e3, 2.0), ([E_SP + (0.001,)], 1e4, 5.0)]
    x = [_crossing(sp, g, k, 12.0)[0] for sp, g, k in sets]
    assert max(x) - min(x) <= 0.05 / xi_transition(1.0, 12.0) + 1e-12, x


def test_boundary_tends_to_xi_tr(oracle):
    """Sec. III.B: the asymptotic (Gamma_CFI tau >> 1) boundary sits at xi_tr.  The measured
    boundary lies behind xi_tr and closes in on it as Gamma_CFI tau doubles (1.73, 1.50, 1.33
    xi_tr at 10, 20, 40); ahead of it the first full window is magnetically dominated."""
    sp, g, k = [E_SP + (0.01,)], 1e3, 2.0
    runs = [_crossing(sp, g, k, gt) for gt in (10.0, 20.0, 40.0)]
    x = [r[0] for r in runs]
    assert all(v > 1.0 for v in x) and x[0] > x[1] > x[2] and x[2] < 1.4, x
    for _, R in runs:
        valid = R[~np.isnan(R)]
        assert valid[0] < 0.0
