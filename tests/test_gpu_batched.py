"""GPU parity of the batched, xi-segmented launch (many instances in one persistent kernel,
each 64-lane block of modes split into xi-segments that pass the oscillator carries to each
other) against the FP64 oracle, and against the unsegmented launch.

Bars as for the single-instance path: FP64 |d ln| <= 1e-9, FP32 |d ln A| <= 1e-4.
"""
import numpy as np
import pytest

from helpers import fields_compare, ln_compare, mode_k, oracle_beam, oracle_run

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
FP32_TOL = 1e-4


def _slab(**kw):
    from paper_2607_24234_amd import inputs
    d = inputs.slab()
    d.update(kw)
    return d


def _views(s, out, i):
    return (s.snapshot_view(out["ln_e"], i).cpu().numpy(), s.snapshot_view(out["ln_b"], i).cpu().numpy())


@pytest.mark.parametrize("precision,amp", [(0, 3e6), (1, 3e29)])
@pytest.mark.parametrize("seg", [1, 7, 37, 299])
def test_segmented_matches_oracle(qs, precision, amp, seg):
    """One instance split into segments of `seg` cells (ragged last segment; the segment count
    is capped by the workgroup size), seeded next to the top of the renormalization range so
    that segments of one mode change scale at different steps."""
    inst = _slab(n_xi=300, length=30.0, kx=np.linspace(0.05, 4.0, 45), seed_amp=amp, d_tau=40.0)
    s = qs.Solver([inst], precision=precision, segment_cells=seg)
    pl = s.plan()
    cap = 12 if precision == qs.QS_FP32 else 8   # waves per workgroup of the march kernel
    assert pl["max_segments"] == min(cap, -(-300 // seg))
    n = 24
    out = s.step(n, out_every=4, snapshots=True, max_ln_a=True)
    fin = s.step(0, snapshots=True)
    s.sync_check()
    ln_e, ln_b, mx, st = oracle_run(inst, n, out_every=4)
    tol = FP64_TOL if precision == qs.QS_FP64 else FP32_TOL
    ge, gb = _views(s, out, 0)
    fields_compare(ge, gb, ln_e, ln_b, tol, what="seg", per_field_ln=precision == qs.QS_FP64)
    ln_compare(out["max_ln_a"].cpu().numpy(), mx, tol, what="seg max ln A")
    import oracle as O
    fe, fb, _ = O.run(oracle_beam(inst), mode_k(inst), inst["d_tau"], 0, st)
    fields_compare(*_views(s, fin, 0), fe, fb, tol, what="seg final", per_field_ln=precision == qs.QS_FP64)
    # the canonical state agrees with the oracle's (per-segment scales folded in exactly)
    cs = s.get_state()[0]
    beam = oracle_beam(inst)
    for m in (0, 22, 44):
        rho, _, _ = O.collapse(beam, st, m)
        g = cs["rho"][m] * 2.0 ** cs["log2_scale"][m]
        assert np.max(np.abs(g - rho)) <= (1e-9 if precision == qs.QS_FP64 else 1e-4) * np.max(np.abs(rho))


@pytest.mark.parametrize("precision", [0, 1])
def test_segmented_equals_unsegmented(qs, precision):
    """The segmented launch reproduces the unsegmented one: the scales are exact powers of
    two, so the arithmetic is the same up to the rounding of the log shift."""
    inst = _slab(n_xi=200, length=25.0, kx=np.linspace(0.1, 3.0, 40), d_tau=30.0)
    a = qs.Solver([inst], precision=precision, segment_cells=1 << 20)
    b = qs.Solver([inst], precision=precision, segment_cells=13)
    assert a.plan()["max_segments"] == 1 and b.plan()["max_segments"] > 1
    ra = a.step(20, out_every=5, snapshots=True, max_ln_a=True)
    rb = b.step(20, out_every=5, snapshots=True, max_ln_a=True)
    tol = 1e-12 if precision == qs.QS_FP64 else 2e-6
    for key in ("ln_e", "ln_b", "max_ln_a"):
        x, y = ra[key].cpu().numpy(), rb[key].cpu().numpy()
        assert np.array_equal(np.isfinite(x), np.isfinite(y))
        f = np.isfinite(x)
        assert np.max(np.abs(x[f] - y[f])) <= tol, key
    a.sync_check()
    b.sync_check()


def test_segmented_deterministic(qs):
    """Per-step maxima of a mode's segments combine by integer atomic max of order-preserving
    keys, so repeated runs are bitwise equal."""
    from paper_2607_24234_amd import inputs
    insts = inputs.batched(n_instances=12, n_modes=40, n_steps=8, max_cells=700)
    r = []
    for _ in range(2):
        s = qs.Solver(insts, precision=qs.QS_FP32, segment_cells=50)
        r.append(s.step(8, out_every=4, snapshots=True, max_ln_a=True))
        s.sync_check()
    for key in ("ln_e", "ln_b", "max_ln_a"):
        assert np.array_equal(r[0][key].cpu().numpy(), r[1][key].cpu().numpy())


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_auto_plan_matches_oracle(qs, precision):
    """The batched sweep at reduced size (24 instances x 70 modes, 128..900 cells) with the
    automatic plan: instances with one and with many segments share one launch."""
    from paper_2607_24234_amd import inputs
    n_steps = 12
    insts = inputs.batched(n_instances=24, n_modes=70, n_steps=n_steps, max_cells=900)
    s = qs.Solver(insts, precision=precision)
    out = s.step(n_steps, out_every=6, snapshots=True, max_ln_a=True)
    s.sync_check()
    mx_all = out["max_ln_a"].cpu().numpy()
    tol = FP64_TOL if precision == qs.QS_FP64 else FP32_TOL
    for i in range(0, 24, 3):
        ln_e, ln_b, mx, _ = oracle_run(insts[i], n_steps, out_every=6, instance=i)
        ge, gb = _views(s, out, i)
        fields_compare(ge, gb, ln_e, ln_b, tol, what="batched %d" % i, per_field_ln=precision == qs.QS_FP64)
        ln_compare(mx_all[:, 70 * i:70 * (i + 1)], mx, tol, what="batched max %d" % i)


def test_batched_full_size_sampled(qs):
    """The batched sweep at full size (256 instances x 128 modes, 128..8192 cells, 200
    steps, FP32 state) in the automatic plan; sampled (instance, mode) pairs against the
    oracle, every step's max ln A."""
    import torch
    from paper_2607_24234_amd import inputs
    insts = inputs.batched()
    assert len(insts) == 256 and min(i["n_xi"] for i in insts) >= 128 and max(i["n_xi"] for i in insts) <= 8192
    s = qs.Solver(insts, precision=qs.QS_FP32)
    assert s.plan()["max_segments"] > 1
    n_steps = insts[0]["n_steps"]
    out = s.step(n_steps, max_ln_a=True)
    torch.cuda.synchronize()
    s.sync_check()
    mx_all = out["max_ln_a"].cpu().numpy()
    assert np.all(np.isfinite(mx_all))
    lens = np.array([i["n_xi"] for i in insts])
    pick = sorted({int(np.argmax(lens)), int(np.argmin(lens)), 0, 97, 200})
    for i in pick:
        modes = np.array([0, 1, 63, 127])
        _, _, mx, _ = oracle_run(insts[i], n_steps, modes=modes, instance=i, n_threads=4)
        ln_compare(mx_all[:, 128 * i + modes], mx, FP32_TOL, what="batched full max %d" % i)


def test_plan_arguments(qs):
    inst = _slab(n_xi=64, kx=np.array([1.0]))
    with pytest.raises(qs.QSError):
        qs.Solver([inst], precision=qs.QS_FP32, columns_per_lane=3)
    with pytest.raises(qs.QSError):
        qs.Solver([inst], precision=qs.QS_FP32, segment_cells=-1)
    for nc in (1, 2):
        s = qs.Solver([inst], precision=qs.QS_FP32, columns_per_lane=nc, segment_cells=16)
        p = s.plan()
        assert p["columns_per_lane"] == nc and p["max_segments"] == 4 and p["workgroups"] == 1


def test_graph_replays_match_eager(qs):
    """A captured 7-step call replayed three times, with eager work and synchronizations in
    between, gives bitwise the outputs of three eager 7-step calls."""
    import torch
    from paper_2607_24234_amd import inputs
    insts = inputs.batched(n_instances=6, n_modes=40, n_steps=21, max_cells=400)
    a = qs.Solver(insts, precision=qs.QS_FP32, segment_cells=60)
    b = qs.Solver(insts, precision=qs.QS_FP32, segment_cells=60)
    g = qs.Graph(b, 7, out_every=3, snapshots=True, max_ln_a=True)
    for rep in range(3):
        ra = a.step(7, out_every=3, snapshots=True, max_ln_a=True)
        rb = g.replay()
        torch.cuda.synchronize()
        for key in ("ln_e", "ln_b", "max_ln_a"):
            assert np.array_equal(ra[key].cpu().numpy(), rb[key].cpu().numpy()), (rep, key)
        x = torch.randn(1000, device="cuda").sum()  # unrelated eager work between replays
        assert torch.isfinite(x)
    assert b.steps_done == 21
    b.sync_check()
    g.close()


def test_tuner_and_cache(qs, tmp_path, monkeypatch):
    from paper_2607_24234_amd import inputs
    insts = inputs.batched(n_instances=10, n_modes=70, n_steps=20, max_cells=1500)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("QS_TUNE_CACHE", str(cache))
    t1 = qs.tune(insts, qs.QS_FP32, steps_per_call=20)
    assert t1["columns_per_lane"] in (1, 2) and t1["segment_cells"] > 0 and t1["ms_per_step"] > 0
    assert len(cache.read_text().splitlines()) == 1
    t2 = qs.tune(insts, qs.QS_FP32, steps_per_call=20)
    assert t2 == t1 and len(cache.read_text().splitlines()) == 1  # served from the cache
    # the tuned plan is a valid plan: parity against the oracle on two instances
    s = qs.Solver(insts, precision=qs.QS_FP32, columns_per_lane=t1["columns_per_lane"],
                  segment_cells=t1["segment_cells"])
    out = s.step(20, max_ln_a=True)
    s.sync_check()
    mx_all = out["max_ln_a"].cpu().numpy()
    for i in (0, 7):
        _, _, mx, _ = oracle_run(insts[i], 20, instance=i)
        ln_compare(mx_all[:, 70 * i:70 * (i + 1)], mx, FP32_TOL, what="tuned %d" % i)


@pytest.mark.parametrize("precision", [0, 1])
def test_aligned_snapshot_rows_equal_dense(qs, precision):
    """qs_set_snapshot_align: two instances with odd mode counts, their snapshot rows padded to
    32 modes, give bitwise the dense layout's values at every snapshot (only the addresses
    change), leave the padding unwritten and the per-step maxima unchanged; the call is
    refused while a graph of the context exists."""
    import torch
    insts = [_slab(n_xi=150, length=20.0, kx=np.linspace(0.1, 3.0, 45), d_tau=30.0),
             _slab(n_xi=97, length=12.0, kx=np.linspace(0.2, 2.5, 70), d_tau=25.0)]
    a = qs.Solver(insts, precision=precision, segment_cells=40)
    b = qs.Solver(insts, precision=precision, segment_cells=40)
    b.set_snapshot_align(32)
    assert b.snap_ld == [64, 96] and b.snap_elems == 150 * 64 + 97 * 96
    n, every = 12, 4
    ra = a.step(n, out_every=every, snapshots=True, max_ln_a=True)
    out = {k: torch.full((n // every, b.snap_elems), float("nan"), dtype=b.dtype, device="cuda")
           for k in ("ln_e", "ln_b")}
    rb = b.step(n, out_every=every, snapshots=True, max_ln_a=True, out=out)
    assert torch.equal(ra["max_ln_a"], rb["max_ln_a"])
    for key in ("ln_e", "ln_b"):
        for i in range(2):
            x, y = a.snapshot_view(ra[key], i), b.snapshot_view(rb[key], i)
            assert x.shape == y.shape and torch.equal(x, y)
            off = sum(ld * m for ld, m in zip(b.snap_ld[:i], b.n_xi[:i]))
            rows = rb[key][:, off:off + b.n_xi[i] * b.snap_ld[i]].reshape(n // every, b.n_xi[i], b.snap_ld[i])
            assert bool(torch.isnan(rows[..., b.n_modes[i]:]).all())
    # a graph made on the aligned context writes the aligned layout on every replay: the same
    # values as eager aligned steps from the same state; the layout cannot change under it
    c = qs.Solver(insts, precision=precision, segment_cells=40)
    c.set_snapshot_align(32)
    c.step(n)
    g = qs.Graph(b, 4, out_every=2, snapshots=True, max_ln_a=True)
    with pytest.raises(qs.QSError) as e:
        b.set_snapshot_align(1)
    assert e.value.status == qs.QS_ERR_STATE
    for _ in range(2):
        rg = g.replay()
        torch.cuda.synchronize()
        rc = c.step(4, out_every=2, snapshots=True, max_ln_a=True)
        for key in ("ln_e", "ln_b", "max_ln_a"):
            assert torch.equal(rg[key], rc[key]) if key == "max_ln_a" else all(
                torch.equal(b.snapshot_view(rg[key], i), c.snapshot_view(rc[key], i)) for i in range(2))
    g.close()
    b.set_snapshot_align(1)
    assert b.snap_elems == a.snap_elems
