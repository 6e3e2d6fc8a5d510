"""FP64 CPU oracle of the E/B regime diagnostic -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU baseline may import this module.

Sec. III.C tells the two instability regimes of a beam seeded at its front apart by which
field carries more energy at a position: the magnetic field in the spatiotemporal-CFI region
near the front, the electric field in the spatiotemporal-OTSI region behind it, the energies
being taken over a longitudinal window of one skin depth on either side of the position.
Sec. III.B places the boundary at xi_tr = 2 Gamma_CFI tau / sqrt(27), the same in
(xi, Gamma_CFI tau) for every beam-plasma parameter set (Fig. 1).

For one transverse mode with fields on cells j = 0 .. N-1 (ln|E|, ln|B| per cell, as the
solver's snapshots give them) this module computes the plain definition

    R_j = 1/2 ln( sum_{|i-j| <= w} |E_i|^2  /  sum_{|i-j| <= w} |B_i|^2 ),   w <= j < N - w,

NaN where the window would leave the cells, and the first cell j from the front with
R_j > 0 (-1 if there is none): the measured start of the electrically dominated region.
Each field's window sum is taken relative to that field's largest value in the window (FP64),
so fields spanning many decades along xi, or far apart from each other, lose nothing.
"""
from __future__ import annotations

import numpy as np


def log_ratio_map(ln_e, ln_b, w):
    """R [n_xi][n_modes] (float64) from ln|E|, ln|B| laid out [n_xi][n_modes]; half-window w
    cells (the window holds 2 w + 1 cells)."""
    ln_e = np.asarray(ln_e, np.float64)
    ln_b = np.asarray(ln_b, np.float64)
    if ln_e.ndim == 1:
        ln_e, ln_b = ln_e[:, None], ln_b[:, None]
    n = ln_e.shape[0]
    out = np.full(ln_e.shape, np.nan)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for j in range(w, n - w):
            out[j] = _log_energy(ln_e[j - w:j + w + 1]) - _log_energy(ln_b[j - w:j + w + 1])
    return out


def _log_energy(v):
    """1/2 ln sum_i e^{2 v_i} down axis 0, relative to the largest v (NaN if a v is NaN,
    -inf if every v is -inf)."""
    top = v.max(axis=0)
    safe = np.where(np.isneginf(top), 0.0, top)
    s = np.exp(2.0 * (v - safe)).sum(axis=0)
    return np.where(np.isneginf(top), -np.inf, safe + 0.5 * np.log(s))


def first_e_cell(R):
    """Per mode, the first cell j with R_j > 0, or -1 (int64 [n_modes])."""
    R = np.asarray(R, np.float64)
    if R.ndim == 1:
        R = R[:, None]
    hit = R > 0.0
    first = np.argmax(hit, axis=0)
    return np.where(hit.any(axis=0), first, -1).astype(np.int64)


def half_window_cells(half_width, h):
    """Cells within half_width of a cell centre on either side: floor(half_width / h), with a
    relative allowance of 1e-9 for a ratio that is an integer up to rounding."""
    return int(np.floor(half_width / h * (1.0 + 1e-9)))
