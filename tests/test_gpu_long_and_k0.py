"""GPU parity at the lengths the benchmark runs, and of the k = 0 (two-stream) mode.

- the k = 0 mode in a mode list, noise seed, FP64 (1e-9) and FP32 (1e-4), and its exact
  response to a charge impulse (Sec. IV.A) on the GPU state;
- the 3D spectral workload (205,859 modes x 4096 cells) in FP32 for all 2000 steps with the
  launch plan the benchmark's autotuner picks (one column per lane, 1024-cell segments):
  per-step max ln A and the four snapshots of 16 sampled modes, including k = 0 and the
  largest |k|, against the FP64 oracle; and in FP64 for 200 steps;
- the finite-width path over 8192 cells against the grid oracle.
"""
import math

import numpy as np
import pytest

import oracle as O
from helpers import fields_compare, ln_compare, oracle_beam, oracle_run

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
FP32_TOL = 1e-4


def _k0_inst(**kw):
    from paper_2607_24234_amd import inputs
    kx = np.array([0.0, 0.4, -0.3, 0.0, 2.0])
    ky = np.array([0.0, 0.0, 0.3, 0.05, 1.0])
    d = dict(species=[inputs.ELECTRON + (0.1,)], gamma=10.0, length=30.0, n_xi=300, kx=kx, ky=ky,
             d_tau=5.0, seed_kind=inputs.SEED_NOISE, seed_amp=1e-6, rng_seed=4)
    d.update(kw)
    return d


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_k0_mode_parity(qs, precision):
    """A mode list holding k = 0 beside small and large |k|: at k = 0 only the gamma^-3
    longitudinal current couples beam and plasma (E_perp = B_perp = 0, ln|B| = -inf)."""
    inst = _k0_inst()
    prec = qs.QS_FP64 if precision == "fp64" else qs.QS_FP32
    n, every = 60, 10
    s = qs.Solver([inst], precision=prec)
    out = s.step(n, out_every=every, snapshots=True, max_ln_a=True)
    s.sync_check()
    ge = s.snapshot_view(out["ln_e"]).cpu().numpy()
    gb = s.snapshot_view(out["ln_b"]).cpu().numpy()
    gm = out["max_ln_a"].cpu().numpy()
    ln_e, ln_b, mx, _ = oracle_run(inst, n, out_every=every)
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    fields_compare(ge, gb, ln_e, ln_b, tol, what="k0", per_field_ln=precision == "fp64")
    ln_compare(gm, mx, tol, what="k0 max ln A")
    assert np.all(np.isneginf(gb[:, :, 0])) and np.all(np.isfinite(ge[:, :, 0]))
    # the k = 0 mode does evolve under the longitudinal coupling
    assert abs(mx[-1, 0] - mx[0, 0]) > 0.05


def test_k0_charge_impulse_exact_gpu(qs):
    """A charge impulse rho = 1/h in cell 0 at k = 0, set through qs_set_state (Sec. IV.A):
    the GPU's fields follow the oracle to 1e-9, and |E_par| = |d_xi n_p| follows the
    xi-derivative of the exact Laplace-form response (exact_refs) at the impulse-centred
    positions to the discretization's second-order error at 256 cells."""
    from exact_refs import charge_impulse_series
    from paper_2607_24234_amd import inputs
    nb, g, L, N, dt, T = 0.1, 10.0, 8.0, 256, 1.0, 300.0
    beta = math.sqrt(nb / g ** 3)
    h = L / N
    inst = dict(species=[inputs.ELECTRON + (nb,)], gamma=g, length=L, n_xi=N, kx=np.array([0.0]), ky=None,
                d_tau=dt, seed_kind=4, seed_amp=1.0, rng_seed=0)
    s = qs.Solver([inst], precision=qs.QS_FP64)
    z = np.zeros((1, N), np.complex128)
    rho = z.copy()
    rho[0, 0] = 1.0 / h
    s.set_state([{"rho": rho, "j_par": z, "j_perp": z, "log2_scale": np.zeros(1)}])
    n = int(round(T / dt))
    s.step(n)
    fin = s.step(0, snapshots=True)
    s.sync_check()
    ge = s.snapshot_view(fin["ln_e"]).cpu().numpy()[0, :, 0]
    # the oracle from the same state
    beam = oracle_beam(inst)
    st = O.ModeState.zeros(1, beam)
    st.n[0, 0, 0] = (1.0 / h) / inputs.ELECTRON[0]
    O.run(beam, [0.0], dt, n, st, want_fields=False, want_max=False)
    f = O.mode_fields(beam, 0.0, st)
    m = f["ln_e"] > np.max(f["ln_e"]) + math.log(1e-6)
    assert np.max(np.abs(ge[m] - f["ln_e"][m])) <= FP64_TOL
    # |E_par| = |d_xi n_p| against the exact response's xi-derivative (central difference)
    idx = np.arange(8, N - 8, 16)
    eps = 1e-4
    ref = np.array([abs(charge_impulse_series(T, (j + 0.5) * h - h / 2 + eps, 0.0, beta) -
                        charge_impulse_series(T, (j + 0.5) * h - h / 2 - eps, 0.0, beta)) / (2 * eps) for j in idx])
    got = np.exp(ge[idx])
    assert np.max(np.abs(got - ref)) / np.max(ref) < 3e-4


def _sample_3d(kx, ky):
    """16 modes of the 3D list: k = 0, the four largest |k|, a few in between, and random ones."""
    k = np.hypot(kx, ky)
    zero = int(np.flatnonzero(k == 0.0)[0])
    order = np.argsort(k)
    rng = np.random.default_rng(7)
    pick = [zero, order[-1], order[-2], order[-3], order[-4], order[len(k) // 2], order[len(k) // 4],
            int(np.argmin(np.abs(k - 1.0))), int(np.argmin(np.abs(k - 3.0))), 0, len(k) - 1]
    pick += list(rng.integers(0, len(k), 16))
    out = []
    for p in pick:
        if int(p) not in out:
            out.append(int(p))
    return np.array(sorted(out[:16]))


def test_spectral3d_headline_fp32_all_steps(qs):
    """The benchmark's workload and plan for its whole length: 2000 steps of FP32 state with
    FP64 carries, one column per lane in 1024-cell segments (the autotuner's pick), snapshots
    every 500 steps; 16 sampled modes against the FP64 oracle (renormalized, the run grows by
    ~93 nepers)."""
    import torch
    from paper_2607_24234_amd import inputs
    inst = inputs.spectral3d()
    kx, ky = inst["kx"], inst["ky"]
    sample = _sample_3d(kx, ky)
    assert np.hypot(kx, ky)[sample].min() == 0.0 and np.hypot(kx, ky)[sample].max() > 5.99
    n, every = 2000, 500
    s = qs.Solver([inst], precision=qs.QS_FP32, columns_per_lane=1, segment_cells=1024)
    assert s.plan()["max_segments"] == 4
    out = s.step(n, out_every=every, snapshots=True, max_ln_a=True)
    idx = torch.as_tensor(sample, device="cuda")
    gm = out["max_ln_a"][:, idx].cpu().numpy()
    ge = s.snapshot_view(out["ln_e"])[:, :, idx].cpu().numpy()
    gb = s.snapshot_view(out["ln_b"])[:, :, idx].cpu().numpy()
    del out
    torch.cuda.synchronize()
    s.sync_check()
    ln_e, ln_b, mx, _ = oracle_run(inst, n, out_every=every, modes=sample, renorm=True)
    assert np.max(mx[-1] - mx[0]) > 80.0
    ln_compare(gm, mx, FP32_TOL, what="3d 2000-step max ln A")
    fields_compare(ge, gb, ln_e, ln_b, FP32_TOL, what="3d 2000 steps")
    s.close()


def test_spectral3d_twenty_step_call_aligned(qs):
    """The benchmark's short form: 5 steps, then one call of 20 steps whose first step writes
    the snapshot into rows aligned to 32 modes, with the autotuner's plan for 20-step calls (2
    segments of 2048 cells); 16 sampled modes of the per-step maxima and of the snapshot (the
    state after 5 steps) against the FP64 oracle."""
    import torch
    from paper_2607_24234_amd import inputs
    inst = inputs.spectral3d()
    sample = _sample_3d(inst["kx"], inst["ky"])
    s = qs.Solver([inst], precision=qs.QS_FP32, columns_per_lane=1, segment_cells=2048)
    s.set_snapshot_align(32)
    assert s.plan()["max_segments"] == 2 and s.snap_elems == inst["n_xi"] * 205888
    idx = torch.as_tensor(sample, device="cuda")
    warm = s.step(5, max_ln_a=True)
    out = s.step(20, out_every=20, snapshots=True, max_ln_a=True)
    gm = torch.cat([warm["max_ln_a"], out["max_ln_a"]])[:, idx].cpu().numpy()
    ge = s.snapshot_view(out["ln_e"])[:, :, idx].cpu().numpy()
    gb = s.snapshot_view(out["ln_b"])[:, :, idx].cpu().numpy()
    del out, warm
    torch.cuda.synchronize()
    s.sync_check()
    ln_e, ln_b, mx, _ = oracle_run(inst, 25, out_every=5, modes=sample, renorm=True)
    ln_compare(gm, mx, FP32_TOL, what="3d 20-step call max ln A")
    fields_compare(ge, gb, ln_e[1:2], ln_b[1:2], FP32_TOL, what="3d 20-step call snapshot")
    s.close()


def test_spectral3d_fp64_200_steps(qs):
    """The same workload in FP64 for 200 steps (three 1366-cell segments), snapshots every
    100 steps: 16 sampled modes to 1e-9."""
    import torch
    from paper_2607_24234_amd import inputs
    inst = inputs.spectral3d()
    sample = _sample_3d(inst["kx"], inst["ky"])
    n, every = 200, 100
    s = qs.Solver([inst], precision=qs.QS_FP64, columns_per_lane=1, segment_cells=1366)
    out = s.step(n, out_every=every, snapshots=True, max_ln_a=True)
    idx = torch.as_tensor(sample, device="cuda")
    gm = out["max_ln_a"][:, idx].cpu().numpy()
    ge = s.snapshot_view(out["ln_e"])[:, :, idx].cpu().numpy()
    gb = s.snapshot_view(out["ln_b"])[:, :, idx].cpu().numpy()
    del out
    torch.cuda.synchronize()
    s.sync_check()
    ln_e, ln_b, mx, _ = oracle_run(inst, n, out_every=every, modes=sample, renorm=True)
    ln_compare(gm, mx, FP64_TOL, what="3d fp64 max ln A")
    fields_compare(ge, gb, ln_e, ln_b, FP64_TOL, what="3d fp64", per_field_ln=True)
    s.close()


def test_grid_long_xi_matches_oracle(qs):
    """Finite width over the workload's 8192 cells (L = 200, n_b = 0.05, gamma = 2000,
    sigma_r = 0.5) on a 16 x 16 transverse grid over 4 x 4, centroid seed, 2 steps of 2:
    the FP64 oscillator carries over the whole beam against the grid oracle."""
    from paper_2607_24234_amd import inputs
    d = inputs.finite_width(nx=16, ny=16, n_xi=8192, n_steps=2, length=200.0, box=4.0, sigma_r=0.5)
    s = qs.GridSolver(d)
    out = s.step(2, out_every=1, snapshots=True, max_ln_a=True)
    s.sync_check()
    nx, ny, N = d["nx"], d["ny"], d["n_xi"]
    x = (np.arange(nx) - nx // 2) * d["lx"] / nx
    y = (np.arange(ny) - ny // 2) * d["ly"] / ny
    gr = np.exp(-(x[None, :] ** 2 + y[:, None] ** 2) / (2 * d["sigma_r"] ** 2))
    om0 = sum(q * q * nb / m for q, m, nb in d["species"])
    G = O.Grid(nx, ny, N, d["lx"], d["ly"], d["length"] / N, d["gamma"], np.broadcast_to(om0 * gr, (N, ny, nx)).copy())
    ost = O.grid_seed(G, d["seed_kind"], d["seed_amp"], offset=d["centroid_offset"], sigma_r=d["sigma_r"],
                      rng_seed=d["rng_seed"])
    ln_e, ln_b, mx = O.grid_run(G, d["d_tau"], 2, ost, out_every=1)
    # A = (|E|^2 + |B|^2)^(1/2) against the snapshot's largest A (one column per snapshot)
    T = ln_e.shape[0]
    fields_compare(out["ln_e"].cpu().numpy().reshape(T, -1, 1), out["ln_b"].cpu().numpy().reshape(T, -1, 1),
                   ln_e.reshape(T, -1, 1), ln_b.reshape(T, -1, 1), FP32_TOL, what="grid 8192 cells")
    assert np.max(np.abs(out["max_ln_a"].cpu().numpy() - mx)) <= FP32_TOL
    st = s.get_state()
    for key, ref in zip(("rho", "j_par", "j_x", "j_y"), ost.arrays()):
        assert np.max(np.abs(st[key] - ref)) <= FP32_TOL * np.max(np.abs(ref)), key
