"""GPU parity of the E/B regime diagnostic (include/qs_regime.h) against the FP64 oracle
(oracle/regime.py).

Bars: FP64 inputs |dR| <= 1e-9; FP32 inputs (the same values on both sides, widened to FP64
for the oracle) |dR| <= 1e-4 -- the window sums are sums of positive terms, so FP32 leaves
a relative error of a few 1e-7 in each, far below the bar.  The first electrically dominated
cell is an integer decided by the sign of R: it must match the oracle's, unless the oracle's
R lies within the bar of zero at one of the two candidates (then the GPU's choice must be a
valid one: R above minus the bar there and below the bar at every valid cell before it).
End to end (solver snapshot, then the map) each L = 1/2 ln sum |F|^2 is a weighted mean of
its cells' ln values, so R inherits at most twice the solver's ln bar.
"""
import math

import numpy as np
import pytest

from oracle import regime as RG

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-4}


def _fields(n_xi, n_modes, seed, special=False):
    """ln|E|, ln|B| as random walks along xi (steps of 0.4 nepers, offsets of +-30), so that a
    column spans tens of nepers; optional columns of -inf, +inf and NaN values."""
    rng = np.random.default_rng(seed)
    e = np.cumsum(rng.normal(0.0, 0.4, (n_xi, n_modes)), axis=0) + rng.uniform(-30, 30, n_modes)
    b = np.cumsum(rng.normal(0.0, 0.4, (n_xi, n_modes)), axis=0) + rng.uniform(-30, 30, n_modes)
    if special and n_modes >= 6:
        e[:, 0] = -np.inf
        b[:, 1] = -np.inf
        e[:, 2] = -np.inf
        b[:, 2] = -np.inf
        e[n_xi // 2, 3] = np.nan
        b[n_xi // 3, 4] = np.inf
        e[: n_xi // 2, 5] = -np.inf
    return e, b


def _check_first(first_gpu, R_ref, tol):
    first_ref = RG.first_e_cell(R_ref)
    for k in np.nonzero(first_gpu != first_ref)[0]:
        col = R_ref[:, k]
        jg, jr = int(first_gpu[k]), int(first_ref[k])
        near = (jr >= 0 and abs(col[jr]) <= tol) or (jg >= 0 and abs(col[jg]) <= tol)
        assert near, "mode %d: first cell %d, oracle %d" % (k, jg, jr)
        before = col[:jg] if jg >= 0 else col
        assert np.all(~(before > tol)), "mode %d: an earlier cell is clearly electric" % k
        if jg >= 0:
            assert col[jg] > -tol


def _compare(qs, e, b, w, precision):
    import torch
    dt = torch.float64 if precision == "fp64" else torch.float32
    te = torch.as_tensor(e, dtype=dt, device="cuda").contiguous()
    tb = torch.as_tensor(b, dtype=dt, device="cuda").contiguous()
    R, F = qs.regime_map(te, tb, w)
    R = R.cpu().numpy().astype(np.float64)
    F = F.cpu().numpy()
    ref = RG.log_ratio_map(te.cpu().numpy().astype(np.float64), tb.cpu().numpy().astype(np.float64), w)
    tol = TOL[precision]
    assert np.array_equal(np.isnan(R), np.isnan(ref)), "NaN pattern differs"
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(R), fin) and np.array_equal(R[~fin & ~np.isnan(ref)], ref[~fin & ~np.isnan(ref)])
    err = float(np.max(np.abs(R[fin] - ref[fin]))) if fin.any() else 0.0
    assert err <= tol, "max |dR| = %.3e" % err
    _check_first(F, ref, tol)
    return R, F


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n_modes,n_xi,w", [(1, 1, 0), (37, 100, 0), (37, 100, 3), (70, 257, 8), (130, 300, 25),
                                             (65, 40, 19), (65, 40, 20), (5, 50, 100), (300, 211, 40),
                                             (64, 300, 50), (50, 300, 90), (40, 400, 130)])
def test_regime_map_matches_oracle(qs, precision, n_modes, n_xi, w):
    """Every form of the kernel: FP32 windows of 8..64 cells stream through the LDS ring
    (several chunks, ragged last chunk, 64-mode blocks partly empty, outputs split over
    workgroups with the first cell combined across them); narrow windows (w < 8, summed
    directly), FP64 windows up to 44 cells and FP32 ones of 65..120 stage tiles in LDS;
    wider ones (w = 50, 90 in FP64, 130 in both) take the one-lane-per-mode form.  Also
    exactly one valid cell (n = 2w + 2), none, and a window longer than the cells."""
    e, b = _fields(n_xi, n_modes, seed=n_modes * 1000 + n_xi + w, special=True)
    _compare(qs, e, b, w, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_windows_far_below_the_span_maximum(qs, precision):
    """A spike 60 nepers above a flat field: the windows of its tiles that do not hold it sum
    to less than exp(-120) relative to the span's largest value and are summed again over
    their own window."""
    n, m, w = 200, 8, 12
    e = np.zeros((n, m))
    b = np.full((n, m), -0.5)
    for k in range(m):
        e[50 + 7 * k, k] = 60.0
        b[120 + 5 * k, k] = 80.0
    _compare(qs, e, b, w, precision)


@pytest.mark.parametrize("slope", [-0.3, 0.3, -0.05])
def test_steep_fields_across_chunks(qs, slope):
    """Fields falling (or rising) by 0.3 or 0.05 nepers per cell, with noise: across the
    streaming form's 128-output chunks the span maximum moves by up to ~40 nepers, so the
    windows far below a chunk's reference (summed again from memory) and the chunk-to-chunk
    hand-over of the halo rows are both exercised; FP32 against the oracle."""
    n_xi, n_modes, w = 1000, 70, 40
    rng = np.random.default_rng(int(abs(slope) * 100) + (slope > 0))
    j = np.arange(n_xi)[:, None]
    e = slope * j + rng.normal(0, 0.3, (n_xi, n_modes)) + rng.uniform(-5, 5, n_modes)
    b = slope * j + rng.normal(0, 0.3, (n_xi, n_modes)) + rng.uniform(-5, 5, n_modes)
    _compare(qs, e, b, w, "fp32")


def test_outputs_optional_and_argument_errors(qs):
    import torch
    e, b = _fields(64, 10, seed=3)
    te = torch.as_tensor(e, device="cuda")
    tb = torch.as_tensor(b, device="cuda")
    R, F = qs.regime_map(te, tb, 5, first_e_cell=False)
    assert F is None and R is not None
    R2, F2 = qs.regime_map(te, tb, 5, log_ratio=False)
    assert R2 is None
    assert np.array_equal(F2.cpu().numpy(), RG.first_e_cell(R.cpu().numpy()))
    L = qs.lib()
    assert L.qs_regime_map(qs._vp(te), qs._vp(tb), 10, 64, 5, 1, None, None, None) == qs.QS_ERR_ARG
    assert L.qs_regime_map(qs._vp(te), qs._vp(tb), 10, 64, 5, 7, qs._vp(R), None, None) == qs.QS_ERR_ARG
    assert L.qs_regime_map(qs._vp(te), qs._vp(tb), 0, 64, 5, 0, qs._vp(R), None, None) == qs.QS_ERR_ARG
    assert L.qs_regime_map(qs._vp(te), qs._vp(tb), 10, 64, -1, 0, qs._vp(R), None, None) == qs.QS_ERR_ARG
    assert L.qs_regime_map(None, qs._vp(tb), 10, 64, 5, 0, qs._vp(R), None, None) == qs.QS_ERR_ARG


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_regime_of_solver_snapshot(qs, precision):
    """End to end: a pair beam (n_b = 0.02 per species, gamma = 2e4) seeded at its front, four
    modes k = 2..5 run to Gamma_CFI(3) tau = 12 by the GPU solver, its final ln|E|, ln|B|
    snapshot through the GPU map (one skin depth either side), against the oracle solver's
    fields through the oracle map.  The measured boundary sits behind xi_tr for every mode."""
    import torch
    import oracle as O
    from exact_refs import gamma_cfi, xi_transition
    from helpers import oracle_beam, oracle_run
    from paper_2607_24234_amd import inputs
    sp = [(-1.0, 1.0, 0.02), (1.0, 1.0, 0.02)]
    G3 = gamma_cfi(sp, 2e4, 3.0)
    n, L, n_xi = 400, 24.0, 480
    inst = inputs.slab(n_modes=4, n_xi=n_xi, n_steps=n)
    inst.update(species=sp, gamma=2e4, length=L, kx=np.array([2.0, 3.0, 4.0, 5.0]), d_tau=12.0 / G3 / n,
                seed_kind=O.SEED_FRONT_IMPULSE, seed_amp=1e-6)
    prec = qs.QS_FP64 if precision == "fp64" else qs.QS_FP32
    s = qs.Solver([inst], precision=prec)
    s.step(n)
    f = s.step(0, snapshots=True)
    s.sync_check()
    te = s.snapshot_view(f["ln_e"])[0].contiguous()
    tb = s.snapshot_view(f["ln_b"])[0].contiguous()
    h = L / n_xi
    w = RG.half_window_cells(1.0, h)
    R, F = qs.regime_map(te, tb, w)
    R = R.cpu().numpy().astype(np.float64)
    F = F.cpu().numpy()
    _, _, _, st = oracle_run(inst, n, renorm=True)
    beam = oracle_beam(inst)
    fe = np.empty((n_xi, 4))
    fb = np.empty((n_xi, 4))
    for m, k in enumerate(inst["kx"]):
        d = O.mode_fields(beam, k, st, m)
        fe[:, m], fb[:, m] = d["ln_e"], d["ln_b"]
    ref = RG.log_ratio_map(fe, fb, w)
    tol = 2 * (1e-9 if precision == "fp64" else 1e-4)
    # compare where both fields' window maxima are within 1e-6 of their column maxima (the
    # solver's bar holds there)
    valid = ~np.isnan(ref)
    mask = valid.copy()
    for m in range(4):
        ce, cb = fe[:, m].max(), fb[:, m].max()
        for j in np.nonzero(valid[:, m])[0]:
            mask[j, m] = fe[j - w:j + w + 1, m].max() >= ce - math.log(1e6) and fb[j - w:j + w + 1, m].max() >= cb - math.log(1e6)
    assert mask.sum() > 0.8 * valid.sum()
    err = float(np.max(np.abs(R[mask] - ref[mask])))
    assert err <= tol, "max |dR| = %.3e" % err
    _check_first(F, ref, tol)
    tau = n * inst["d_tau"]
    for m, k in enumerate(inst["kx"]):
        assert F[m] >= 0
        assert (F[m] + 0.5) * h > xi_transition(gamma_cfi(sp, 2e4, k), tau), (k, F[m])


def _sampled_device_fields(n_modes, n_xi, seed):
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    e = torch.cumsum(torch.randn((n_xi, n_modes), device="cuda", generator=g) * 0.4, dim=0)
    e += (torch.rand(n_modes, device="cuda", generator=g) * 60 - 30)[None, :]
    b = torch.cumsum(torch.randn((n_xi, n_modes), device="cuda", generator=g) * 0.4, dim=0)
    b += (torch.rand(n_modes, device="cuda", generator=g) * 60 - 30)[None, :]
    return e.contiguous(), b.contiguous()


def _check_sampled(qs, e, b, w, n_cols):
    import torch
    R, F = qs.regime_map(e, b, w)
    torch.cuda.synchronize()
    n_modes = e.shape[1]
    cols = torch.as_tensor(np.linspace(0, n_modes - 1, n_cols).astype(np.int64), device="cuda")
    ref = RG.log_ratio_map(e[:, cols].cpu().numpy().astype(np.float64), b[:, cols].cpu().numpy().astype(np.float64), w)
    Rs = R[:, cols].cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(Rs), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert float(np.max(np.abs(Rs[ok] - ref[ok]))) <= 1e-4
    _check_first(F[cols].cpu().numpy(), ref, 1e-4)


def test_regime_chunks_split_over_workgroups(qs):
    """44,800 modes x 1000 cells in FP32 (w = 40): the streaming form splits each 64-mode
    block's eight 128-output chunks over three workgroups of three chunks (ring reuse inside a
    workgroup, the first cell combined across them); 128 modes against the oracle."""
    e, b = _sampled_device_fields(44800, 1000, seed=9)
    _check_sampled(qs, e, b, 40, 128)


@pytest.mark.parametrize("n_modes,n_xi", [(64, 70000), (6400, 20000)])
def test_regime_long_columns(qs, n_modes, n_xi):
    """Long columns (70,000 and 20,000 cells, FP32, w = 40): one 64-mode block whose 547 chunks
    go to 547 workgroups, and 100 blocks whose 156 chunks go 8 at a time to 20 workgroups
    each; 64 modes against the oracle."""
    e, b = _sampled_device_fields(n_modes, n_xi, seed=n_xi)
    _check_sampled(qs, e, b, 40, min(n_modes, 64))


def test_regime_full_size_sampled(qs):
    """The 3D workload's snapshot size, 205,859 modes x 4096 cells in FP32, random-walk fields
    made on the device; the window of the 3D run's cell width (one skin depth = 40 cells); 96
    modes spread over the list against the oracle."""
    e, b = _sampled_device_fields(205859, 4096, seed=5)
    _check_sampled(qs, e, b, 40, 96)
    del e, b


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_regime_boundary_over_a_run(qs, precision):
    """The boundary in the (xi, Gamma_CFI tau) plane over one run: the pair beam of Sec. III.C
    (n_b = 0.02 per species, gamma = 2e4, k = 3) seeded at its front, GPU snapshots every
    Gamma_CFI tau = 5 up to 35, each through the GPU map.  The first electrically dominated
    cell of every snapshot equals the oracle's; the boundary moves back as Gamma tau grows,
    stays behind xi_tr = 2 Gamma tau / sqrt(27) and closes in on it (2.07 xi_tr at 5, 1.36 at
    35 in the oracle)."""
    import oracle as O
    from exact_refs import gamma_cfi, xi_transition
    from helpers import oracle_run
    from paper_2607_24234_amd import inputs
    sp = [(-1.0, 1.0, 0.02), (1.0, 1.0, 0.02)]
    G = gamma_cfi(sp, 2e4, 3.0)
    L, n_xi, n, every = 30.0, 600, 1600, 200
    inst = inputs.slab(n_modes=1, n_xi=n_xi, n_steps=n)
    inst.update(species=sp, gamma=2e4, length=L, kx=np.array([3.0]), d_tau=40.0 / G / n,
                seed_kind=O.SEED_FRONT_IMPULSE, seed_amp=1e-6)
    prec = qs.QS_FP64 if precision == "fp64" else qs.QS_FP32
    s = qs.Solver([inst], precision=prec)
    out = s.step(n, out_every=every, snapshots=True)
    s.sync_check()
    le = s.snapshot_view(out["ln_e"])
    lb = s.snapshot_view(out["ln_b"])
    h = L / n_xi
    w = RG.half_window_cells(1.0, h)
    ref_e, ref_b, _, _ = oracle_run(inst, n, out_every=every, renorm=True)
    tol = 2 * (1e-9 if precision == "fp64" else 1e-4)
    ratios = []
    for t in range(le.shape[0]):
        _, F = qs.regime_map(le[t].contiguous(), lb[t].contiguous(), w, log_ratio=False)
        ref = RG.log_ratio_map(ref_e[t], ref_b[t], w)
        _check_first(F.cpu().numpy(), ref, tol)
        j = int(F[0].item())
        if t == 0:
            assert j == -1
            continue
        ratios.append((j + 0.5) * h / xi_transition(G, t * every * inst["d_tau"]))
    assert all(r > 1.0 for r in ratios), ratios
    assert all(a > b for a, b in zip(ratios, ratios[1:])), ratios
    assert ratios[-1] < 1.45, ratios
