"""Test-side glue: run the oracle on an instance dict from paper_2607_24234_amd.inputs and
compare log-field outputs with the GPU path.  (Test infrastructure: imports the oracle.)"""
from __future__ import annotations

import math

import numpy as np

import oracle as O


def oracle_beam(inst):
    n = inst["n_xi"]
    flags = inst.get("flags", 0)
    return O.Beam(inst["species"], inst["gamma"], n, inst["length"] / n,
                  shape=inst.get("profile_table"), flags=flags)


def mode_k(inst):
    kx = np.asarray(inst["kx"], np.float64)
    ky = inst.get("ky")
    return np.abs(kx) if ky is None else np.sqrt(kx * kx + np.asarray(ky, np.float64) ** 2)


def oracle_run(inst, n_steps, out_every=1, modes=None, instance=0, n_threads=0, renorm=False):
    """Seed (same counter-based noise as the GPU) and run the oracle for the given modes.
    Returns (ln_e, ln_b, max_ln_a, state)."""
    beam = oracle_beam(inst)
    k_all = mode_k(inst)
    modes = np.arange(len(k_all)) if modes is None else np.asarray(modes)
    st = O.ModeState.zeros(len(modes), beam)
    for i, m in enumerate(modes):
        s1 = O.seed(beam, [k_all[m]], inst.get("seed_kind", O.SEED_NOISE), inst.get("seed_amp", 1e-6),
                    rng_seed=inst.get("rng_seed", 0), instance=instance,
                    n_modes_total=len(k_all), mode_offset=int(m))
        st.n[i], st.pz[i], st.pt[i] = s1.n[0], s1.pz[0], s1.pt[0]
    ln_e, ln_b, mx = O.run(beam, k_all[modes], inst["d_tau"], n_steps, st, out_every=out_every,
                           renorm=renorm, n_threads=n_threads, front=front_values(beam, st))
    return ln_e, ln_b, mx, st


def front_values(beam, state):
    """The stationary front's n_p per mode: cell 0's charge density sum_s q_s n_s of `state`
    (the seeded state at tau = 0); None unless the beam has the STATIONARY_FRONT flag."""
    if not beam.flags & O.STATIONARY_FRONT:
        return None
    return np.einsum("s,ms->m", beam.q, state.n[:, :, 0])


def ln_compare(gpu, ref, tol, rel_floor=1e-6, what=""):
    """max |gpu - ref| in ln units; asserts it is <= tol and returns it.

    3D arrays are snapshots [snap][cell][mode]: an entry is compared where its amplitude is
    >= rel_floor times the largest amplitude of its own (snapshot, mode) column over the cells
    (the nodes of a field are left out), so every snapshot of a growing run is compared.
    2D arrays are per-step maxima over the cells [step][mode], which have no nodes: every
    finite entry is compared.  Where the oracle's field vanishes (ln = -inf, e.g. B at k = 0)
    the GPU value must vanish too, or lie below the compared range."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    assert ref.ndim in (2, 3), ref.shape
    if ref.ndim == 3:
        colmax = np.max(np.where(np.isfinite(ref), ref, -np.inf), axis=1, keepdims=True)
        floor = colmax + np.log(rel_floor)
        mask = np.isfinite(ref) & (ref >= floor)
    else:
        floor = np.full(ref.shape, np.inf)
        mask = np.isfinite(ref)
    assert np.all(np.isfinite(gpu[mask])), what + ": non-finite GPU values where the oracle is finite"
    zero = np.isneginf(ref)
    if zero.any():
        g0 = gpu[zero]
        lim = np.broadcast_to(floor, ref.shape)[zero]
        assert np.all(np.isneginf(g0) | (g0 < lim)), what + ": GPU field where the oracle's vanishes"
    err = float(np.max(np.abs(gpu[mask] - ref[mask]))) if mask.any() else 0.0
    assert err <= tol, "%s: max |d ln| = %.3e > %.1e" % (what, err, tol)
    return err


def ln_amplitude(ln_e, ln_b):
    """ln A = 1/2 ln(|E|^2 + |B|^2) from ln|E| and ln|B| (either may be -inf)."""
    ln_e = np.asarray(ln_e, np.float64)
    ln_b = np.asarray(ln_b, np.float64)
    top = np.maximum(ln_e, ln_b)
    out = top.copy()
    f = np.isfinite(top)
    out[f] = top[f] + 0.5 * np.log(np.exp(2 * (ln_e[f] - top[f])) + np.exp(2 * (ln_b[f] - top[f])))
    return out


def fields_compare(g_e, g_b, r_e, r_b, tol, rel_floor=1e-6, what="", per_field_ln=False):
    """Snapshot pairs [snap][cell][mode] of ln|E|, ln|B| against the oracle's.

    The bar is on the mode amplitude A = (|E|^2 + |B|^2)^(1/2), which has no nodes (B and
    E_par are in quadrature with n_p): |d ln A| <= tol on every cell whose A is >= rel_floor
    times the largest A of its (snapshot, mode) column.  Each field alone may pass through a
    node, where a relative error is meaningless; there its error is held to the same bar
    relative to the local A: |E_gpu - E_oracle| <= tol A_oracle (likewise B), i.e. the
    floating-point error model of a value computed beside others of magnitude A.
    per_field_ln: also hold ln|E| and ln|B| themselves to tol (ln_compare; for FP64, whose
    rounding leaves even deep nodes far inside the bar)."""
    if per_field_ln:
        ln_compare(g_e, r_e, tol, rel_floor, what=what + " ln|E|")
        ln_compare(g_b, r_b, tol, rel_floor, what=what + " ln|B|")
    la_g = ln_amplitude(g_e, g_b)
    la_r = ln_amplitude(r_e, r_b)
    err_a = ln_compare(la_g, la_r, tol, rel_floor, what=what + " ln A")
    colmax = np.max(np.where(np.isfinite(la_r), la_r, -np.inf), axis=1, keepdims=True)
    mask = np.isfinite(la_r) & (la_r >= colmax + np.log(rel_floor))
    worst = 0.0
    for name, g, r in (("E", g_e, r_e), ("B", g_b, r_b)):
        g = np.asarray(g, np.float64)
        r = np.asarray(r, np.float64)
        d = np.zeros(mask.shape)
        d[mask] = np.abs(np.exp(g[mask] - la_r[mask]) - np.exp(r[mask] - la_r[mask]))
        e = float(np.max(d)) if mask.any() else 0.0
        if e > tol:
            i = np.unravel_index(int(np.argmax(d)), d.shape)
            raise AssertionError("%s %s: |d%s|/A = %.3e > %.1e at (snap, cell, mode) %s, %s/A = %.3e, A/max A = %.3e"
                                 % (what, name, name, e, tol, i, name, math.exp(r[i] - la_r[i]),
                                    math.exp(la_r[i] - colmax[i[0], 0, i[2]])))
        worst = max(worst, e)
    return max(err_a, worst)


def envelope_compare(gpu, ref, tol, half_window, rel_floor=1e-6, what=""):
    """One field's snapshots [snap][cell][mode] (e.g. ln|F_perp|) against the oracle's, with
    the error of each value measured against the field's local envelope, its largest magnitude
    within +-half_window cells: |F_gpu - F_oracle| <= tol env, on cells whose envelope is >=
    rel_floor times the column's maximum (a field oscillating along xi passes through nodes,
    where only such an absolute error is meaningful)."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert gpu.shape == ref.shape and ref.ndim == 3
    n = ref.shape[1]
    env = np.full(ref.shape, -np.inf)
    for j in range(n):
        lo, hi = max(0, j - half_window), min(n, j + half_window + 1)
        env[:, j, :] = np.max(ref[:, lo:hi, :], axis=1)
    colmax = np.max(env, axis=1, keepdims=True)
    mask = np.isfinite(env) & (env >= colmax + np.log(rel_floor))
    d = np.zeros(mask.shape)
    d[mask] = np.abs(np.exp(gpu[mask] - env[mask]) - np.exp(ref[mask] - env[mask]))
    err = float(np.max(d)) if mask.any() else 0.0
    assert err <= tol, "%s: |dF|/envelope = %.3e > %.1e" % (what, err, tol)
    return err


def windowed_log_ratio(ln_e, ln_b, h, xi):
    """1/2 ln( sum |E|^2 / sum |B|^2 ) over the cells within half a plasma wavelength of xi."""
    ln_e = np.asarray(ln_e, np.float64)
    ln_b = np.asarray(ln_b, np.float64)
    n = len(ln_e)
    c = np.arange(n)
    x = (c + 0.5) * h
    m = np.abs(x - xi) <= math.pi
    top = max(np.max(ln_e[m]), np.max(ln_b[m]))
    return 0.5 * math.log(np.sum(np.exp(2 * (ln_e[m] - top))) / np.sum(np.exp(2 * (ln_b[m] - top))))
