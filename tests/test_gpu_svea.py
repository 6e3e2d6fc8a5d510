"""GPU parity of the envelope-approximation variant (include/qs_svea.h) against the FP64
oracle (oracle/svea.py) and the exact impulse response; its place beside the full model.

Bar: FP64 state, |d ln| <= 1e-9 (relative 1e-9) on every entry, as for the spectral path."""
import math

import numpy as np
import pytest

from exact_refs import svea_series
from oracle import svea as S

pytestmark = pytest.mark.gpu
TOL = 1e-9
E = (-1.0, 1.0)
P = (1.0, 1.0)


def _compare(gn, gm, on, om):
    for g, r, what in ((gn, on, "n"), (gm, om, "m")):
        nz = np.abs(r) > 0
        assert np.array_equal(np.abs(g) > 0, nz), what
        err = np.max(np.abs(np.log(np.abs(g[nz])) - np.log(np.abs(r[nz]))))
        ph = np.max(np.abs(np.angle(g[nz] / r[nz])))
        assert err <= TOL and ph <= TOL, (what, err, ph)


@pytest.mark.parametrize("n_xi,n_modes", [(96, 70), (1, 3), (3, 64), (257, 130)])
def test_matches_oracle(qs, n_xi, n_modes):
    sp, gam = [E + (0.02,), P + (0.01,)], 50.0
    k = np.linspace(0.1, 4.0, n_modes)
    L, dt, n = 12.0, 4.0, 25
    s = qs.SVEASolver(sp, gam, k, L, n_xi, dt)
    s.step(10)
    s.step(n - 10)                      # two calls: the state carries over exactly
    gn, gm = s.state()
    a = S.svea_coefficient(sp, gam, k)
    assert np.max(np.abs(qs.svea_coefficients(sp, gam, k) - a)) <= 1e-15 * np.max(np.abs(a))
    _, on, om = S.run(a, n_xi, L / n_xi, dt, n, out_every=10 ** 9)
    _compare(gn, gm, on, om)


def test_calls_of_every_remainder(qs):
    """Calls of 1, 2, 3 and 5 steps (a sweep advances up to four steps at once, so each call
    ends with a shorter sweep of its remainder) against one oracle run of all 11 steps."""
    sp, gam = [E + (0.02,)], 200.0
    k = np.linspace(0.2, 3.0, 65)
    L, n_xi, dt = 10.0, 77, 3.0
    s = qs.SVEASolver(sp, gam, k, L, n_xi, dt)
    for c in (1, 2, 3, 5):
        s.step(c)
    gn, gm = s.state()
    _, on, om = S.run(S.svea_coefficient(sp, gam, k), n_xi, L / n_xi, dt, 11, out_every=10 ** 9)
    _compare(gn, gm, on, om)


def test_envelope_against_exact_series(qs):
    """N = (i/2) n: |N| on the GPU against the exact impulse response at 256 cells."""
    G = 0.02
    sp = [E + (G * G,)]                  # gamma = 1, large k: Gamma^2 = n_b k^2/(1+k^2) ~ G^2
    k = np.array([1e4])
    a = qs.svea_coefficients(sp, 1.0, k)[0]
    s = qs.SVEASolver(sp, 1.0, k, 8.0, 256, 1.25)
    s.step(160)
    ln = s.ln_envelope().cpu().numpy()[:, 0]
    xi = (np.arange(256) + 0.5) * 8.0 / 256
    ref = np.array([abs(svea_series(a, 200.0, x)) / 2 for x in xi])
    # second-order discretization error, relative to the largest value as in the oracle's pin
    assert np.max(np.abs(np.exp(ln) - ref)) / np.max(ref) < 2e-5


def test_rescaling_is_exact(qs):
    """Growth past 2^100 rescales by powers of two: ln|N| still matches the unscaled oracle."""
    sp, gam = [E + (0.5,)], 1.0
    k = np.array([0.5, 2.0, 8.0])
    L, N, dt, n = 40.0, 64, 2.0, 60
    s = qs.SVEASolver(sp, gam, k, L, N, dt)
    s.step(n)
    ln = s.ln_envelope().cpu().numpy()
    assert np.max(s.log2.cpu().numpy()) > 0
    _, on, _ = S.run(S.svea_coefficient(sp, gam, k), N, L / N, dt, n, out_every=10 ** 9)
    ref = np.log(np.abs(on)) - math.log(2.0)
    assert np.max(ref) > 100 * math.log(2.0)
    assert np.max(np.abs(ln - ref)) <= TOL * np.max(np.abs(ref))


def test_beside_the_full_model(qs):
    """Sec. III.B: the envelope equation misses the spatiotemporal CFI near the front but keeps
    the full model's leading growth far behind it.  Full model: the oracle's n_p for a front
    impulse without the gamma^-2 term; envelope: this GPU path.  Growth between Gamma tau = 10
    and 20 at xi = 0.5 differs by more than half, at xi = 40 by less than a tenth."""
    import oracle as O
    G = 0.02
    sp = [E + (G * G,)]                  # Gamma ~ G at large k
    k = 1e4
    L, N = 48.0, 768
    h = L / N
    beam = O.Beam(sp, 1.0, N, h, flags=O.DROP_LONGITUDINAL)
    st = O.seed(beam, [k], O.SEED_FRONT_IMPULSE, 1.0)
    sv = qs.SVEASolver(sp, 1.0, [k], L, N, 2.5)
    full, env = [], []
    for T in (500.0, 1000.0):
        steps = int(round((T - (0 if not full else 500.0)) / 2.5))
        O.run(beam, [k], 2.5, steps, st, want_fields=False, want_max=False)
        sv.step(steps)
        full.append(np.log(np.abs(O.mode_fields(beam, k, st)["np"])))
        env.append(sv.ln_envelope().cpu().numpy()[:, 0])
    xi = (np.arange(N) + 0.5) * h
    for x, lo, hi in ((0.5, 0.5, None), (40.0, None, 0.1)):
        j = int(np.argmin(np.abs(xi - x)))
        gf = full[1][j] - full[0][j]
        ge = env[1][j] - env[0][j]
        rel = abs(ge / gf - 1.0)
        if lo is not None:
            assert rel > lo, (x, gf, ge)
        else:
            assert rel < hi, (x, gf, ge)


def test_argument_errors(qs):
    import ctypes
    L = qs.lib()
    assert L.qs_svea_step(0, 4, 0.1, None, 1.0, 1, None, None, None, None) == qs.QS_ERR_ARG
    s = qs.SVEASolver([E + (0.01,)], 10.0, [1.0], 4.0, 8, 1.0)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.qs_svea_step(1, 8, -1.0, vp(s.a), 1.0, 1, vp(s.n), vp(s.m), vp(s.log2), None) == qs.QS_ERR_ARG
    assert L.qs_svea_step(1, 8, 0.5, vp(s.a), 1.0, -1, vp(s.n), vp(s.m), vp(s.log2), None) == qs.QS_ERR_ARG
    assert L.qs_svea_step(1, 8, 0.5, vp(s.a), 1.0, 0, vp(s.n), vp(s.m), vp(s.log2), None) == qs.QS_OK
