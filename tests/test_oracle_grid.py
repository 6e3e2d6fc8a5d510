"""Pins of the finite-width oracle (oracle/qs_grid_oracle.c): its FFT against numpy's, a single
transverse Fourier mode in a transversely uniform beam against the spectral oracle (which is
pinned to exact solutions in test_oracle_pins.py), zero density, linearity and the mirror
symmetries of the seeds."""
import math

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("ny,nx", [(8, 8), (4, 16), (32, 2), (1, 8)])
def test_fft_matches_library(ny, nx):
    rng = np.random.default_rng(nx * 100 + ny)
    a = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    assert np.max(np.abs(O.fft2(a) - np.fft.fft2(a))) <= 1e-13 * np.sqrt(nx * ny) * np.max(np.abs(a))
    assert np.max(np.abs(O.fft2(O.fft2(a), inverse=True) - a)) <= 1e-14 * 8


def _grid(nx=16, ny=8, n_xi=24, lx=12.0, ly=9.0, L=6.0, nb=0.02, gamma=50.0, sigma_r=0.0, flags=0):
    h = L / n_xi
    x = (np.arange(nx) - nx // 2) * lx / nx
    y = (np.arange(ny) - ny // 2) * ly / ny
    g = np.ones((ny, nx)) if sigma_r <= 0 else np.exp(-(x[None, :] ** 2 + y[:, None] ** 2) / (2 * sigma_r ** 2))
    omega = np.broadcast_to(nb * g, (n_xi, ny, nx)).copy()   # electron beam: q^2 n_b / m = n_b
    return O.Grid(nx, ny, n_xi, lx, ly, h, gamma, omega, flags)


@pytest.mark.parametrize("flags", [0, 1])
def test_single_mode_equals_spectral_oracle(flags):
    """P-9: uniform transverse profile, rho = S cos(k0 . r): the grid solution is the
    spectral solution at |k0| times cos(k0 . r) (rho, j_par) and k0/|k0| sin(k0 . r) (j_perp)."""
    G = _grid(flags=flags)
    x, y = G.coords()
    k0 = np.array([2 * math.pi * 3 / G.lx, 2 * math.pi * 1 / G.ly])
    kk = float(np.hypot(*k0))
    phase = k0[0] * x[None, :] + k0[1] * y[:, None]
    S, dtau, n = 1e-3, 3.0, 12
    st = O.GridState(G)
    st.rho[:] = S * np.cos(phase)[None, :, :]
    ln_e, ln_b, mx = O.grid_run(G, dtau, n, st, out_every=4)
    beam = O.Beam([(-1.0, 1.0, 0.02)], G.gamma, G.n_xi, G.h, flags=flags)
    ms = O.seed(beam, [kk], O.SEED_UNIFORM, S)
    se, sb, smx = O.run(beam, [kk], dtau, n, ms, out_every=4)
    rho_k, jpar_k, jperp_k = O.collapse(beam, ms, 0)
    scale = np.max(np.abs(rho_k))
    assert np.max(np.abs(rho_k.imag)) <= 1e-14 * scale and np.max(np.abs(jperp_k.real)) <= 1e-14 * np.max(np.abs(jperp_k))
    ref_rho = rho_k.real[:, None, None] * np.cos(phase)[None]
    assert np.max(np.abs(st.rho - ref_rho)) <= 1e-10 * scale
    ref_jpar = jpar_k.real[:, None, None] * np.cos(phase)[None]
    assert np.max(np.abs(st.jpar - ref_jpar)) <= 1e-10 * max(np.max(np.abs(jpar_k)), 1e-300) + 1e-300
    # j_perp = Re[jperp_k khat exp(i phase)] = -Im(jperp_k) khat sin(phase)
    amp = -jperp_k.imag[:, None, None] * np.sin(phase)[None]
    jsc = np.max(np.abs(jperp_k))
    assert np.max(np.abs(st.jx - amp * k0[0] / kk)) <= 1e-10 * jsc
    assert np.max(np.abs(st.jy - amp * k0[1] / kk)) <= 1e-10 * jsc
    # fields: the transverse mean of |E|^2 is half the spectral |E|^2 (Parseval)
    for t in range(ln_e.shape[0]):
        e_mean = np.mean(np.exp(2 * ln_e[t]), axis=(1, 2))
        b_mean = np.mean(np.exp(2 * ln_b[t]), axis=(1, 2))
        assert np.max(np.abs(0.5 * np.log(e_mean) - (se[t][:, 0] - 0.5 * math.log(2)))) <= 1e-9
        assert np.max(np.abs(0.5 * np.log(b_mean) - (sb[t][:, 0] - 0.5 * math.log(2)))) <= 1e-9
    # the box maximum of A is attained where the cosine and sine peaks combine: bounded by
    # the spectral |A| and at least its 1/sqrt(2)
    assert np.all(mx <= smx[:, 0] + 1e-9) and np.all(mx >= smx[:, 0] - 0.5 * math.log(2) - 1e-9)


def test_zero_density_is_static():
    G = _grid(nb=0.0, sigma_r=2.0)
    st = O.grid_seed(G, 0, 1e-4, rng_seed=3)
    r0 = st.rho.copy()
    O.grid_run(G, 5.0, 3, st, want_fields=False, want_max=False)
    assert np.array_equal(st.rho, r0) and not np.any(st.jpar) and not np.any(st.jx) and not np.any(st.jy)


def test_linearity_power_of_two():
    G = _grid(sigma_r=1.5)
    a = O.grid_seed(G, 3, 1e-6, offset=1e-3, sigma_r=1.5, rng_seed=1)
    b = O.grid_seed(G, 3, 1e-6, offset=1e-3, sigma_r=1.5, rng_seed=1)
    for v in b.arrays():
        v *= 8.0
    O.grid_run(G, 2.0, 4, a, want_fields=False, want_max=False)
    O.grid_run(G, 2.0, 4, b, want_fields=False, want_max=False)
    for va, vb in zip(a.arrays(), b.arrays()):
        assert np.array_equal(vb, 8.0 * va)


def test_mirror_symmetries():
    """Gaussian profile centred on the grid: the uniform seed stays even in x, the centroid
    (hosing) seed without noise stays odd in x."""
    G = _grid(nx=16, ny=16, lx=8.0, ly=8.0, sigma_r=1.2)
    mirror = (-np.arange(G.nx)) % G.nx                       # x_i -> -x_i
    f = np.ones(G.n_xi)
    ev = O.grid_seed(G, 1, 1e-3, sigma_r=1.2, f=f)
    od = O.grid_seed(G, 3, 0.0, offset=1e-3, sigma_r=1.2, f=f)
    od.rho[:, :, 0] = 0.0   # the column x = -lx/2 is its own mirror image: odd data vanish there
    s0 = np.max(np.abs(od.rho))
    O.grid_run(G, 4.0, 5, ev, want_fields=False, want_max=False)
    O.grid_run(G, 4.0, 5, od, want_fields=False, want_max=False)
    s = np.max(np.abs(ev.rho))
    assert np.max(np.abs(ev.rho - ev.rho[:, :, mirror])) <= 1e-12 * s
    assert np.max(np.abs(ev.jx + ev.jx[:, :, mirror])) <= 1e-12 * np.max(np.abs(ev.jx))
    s = np.max(np.abs(od.rho))
    assert np.max(np.abs(od.rho + od.rho[:, :, mirror])) <= 1e-12 * s
    # the hosing seed grows: the run is not trivial
    assert s > 1.02 * s0


def _random_problem(n=16, n_xi=16, seed=5):
    """A square periodic grid with a random, nowhere-symmetric positive Omega(xi, y, x) and a
    random state."""
    rng = np.random.default_rng(seed)
    omega = 0.02 * (0.5 + rng.random((n_xi, n, n)))
    G = O.Grid(n, n, n_xi, 7.0, 7.0, 0.25, 40.0, omega)
    st = O.GridState(G)
    for v in st.arrays():
        v[...] = 1e-3 * rng.standard_normal(v.shape)
    st.jpar[-1] = 0.0   # the rear face carries no current
    return omega, G, st


def test_transpose_symmetry():
    """x <-> y on a square grid: the problem with Omega and the state transposed (and j_x, j_y
    exchanged) evolves into the transposed solution.  An x/y mix-up anywhere in the transverse
    solve (a k_x where k_y belongs, a wrong stride of the column transform) breaks it."""
    omega, G, a = _random_problem()
    Gt = O.Grid(G.nx, G.ny, G.n_xi, G.lx, G.ly, G.h, G.gamma, omega.transpose(0, 2, 1).copy())
    b = O.GridState(Gt)
    b.rho[...] = a.rho.transpose(0, 2, 1)
    b.jpar[...] = a.jpar.transpose(0, 2, 1)
    b.jx[...] = a.jy.transpose(0, 2, 1)
    b.jy[...] = a.jx.transpose(0, 2, 1)
    ea, ba, ma = O.grid_run(G, 3.0, 4, a)
    eb, bb, mb = O.grid_run(Gt, 3.0, 4, b)
    for x, y in ((a.rho, b.rho), (a.jpar, b.jpar), (a.jx, b.jy), (a.jy, b.jx)):
        assert np.max(np.abs(x.transpose(0, 2, 1) - y)) <= 1e-12 * np.max(np.abs(x))
    assert np.max(np.abs(ea.transpose(0, 1, 3, 2) - eb)) <= 1e-10
    assert np.max(np.abs(ba.transpose(0, 1, 3, 2) - bb)) <= 1e-10
    assert np.max(np.abs(ma - mb)) <= 1e-10
    # the run is not trivial: the state changed
    _, _, c = _random_problem()
    assert np.max(np.abs(a.rho - c.rho)) > 1e-3 * np.max(np.abs(c.rho))


def test_translation_equivariance():
    """Periodic grid: the problem rolled by whole cells in x and y (Omega and the state)
    evolves into the rolled solution."""
    omega, G, a = _random_problem(seed=9)
    sx, sy = 5, 3
    roll = lambda v: np.roll(v, (sy, sx), axis=(-2, -1))
    Gr = O.Grid(G.nx, G.ny, G.n_xi, G.lx, G.ly, G.h, G.gamma, roll(omega).copy())
    b = O.GridState(Gr)
    for vb, va in zip(b.arrays(), a.arrays()):
        vb[...] = roll(va)
    O.grid_run(G, 3.0, 4, a, want_fields=False, want_max=False)
    O.grid_run(Gr, 3.0, 4, b, want_fields=False, want_max=False)
    for va, vb in zip(a.arrays(), b.arrays()):
        assert np.max(np.abs(roll(va) - vb)) <= 1e-12 * np.max(np.abs(va))
