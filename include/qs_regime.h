/*
 * E/B regime diagnostic over the solver's field snapshots.
 *
 * Sec. III.C of the paper tells the two instability regimes of a beam seeded at its front
 * apart by which field carries more energy at a position, each energy taken over a
 * longitudinal window of one skin depth on either side: the magnetic field dominates where
 * spatiotemporal CFI grows (near the front), the electric field where spatiotemporal OTSI
 * grows (behind it).  Sec. III.B puts the boundary at xi_tr = 2 Gamma_CFI tau / sqrt(27),
 * the same in (xi, Gamma_CFI tau) for every beam-plasma parameter set (Fig. 1).
 *
 * For each mode of a snapshot pair ln|E|, ln|B| (the layout qs_step_tau writes for one
 * instance: [n_xi][n_modes], mode fastest) this call computes
 *
 *     R_j = 1/2 ln( sum_{|i-j| <= w} |E_i|^2 / sum_{|i-j| <= w} |B_i|^2 ),   w <= j < n_xi - w,
 *
 * with w = half_window cells (a window of 2 w + 1 cells; for the paper's window of one skin
 * depth, w = floor(1 / h)), NaN where the window would leave the cells, and per mode the first
 * cell j from the front with R_j > 0 (-1 if none), i.e. the measured start of the electrically
 * dominated region.  Each field's window sum is taken relative to a reference inside the
 * window's neighbourhood, so fields spanning any number of decades along xi are handled;
 * a window holding a NaN gives NaN, one where |E| (|B|) vanishes throughout gives -inf (+inf),
 * one where both vanish NaN.  The per-mode log scales of the snapshots cancel in R.
 *
 * Arguments (device memory, caller-owned):
 *   ln_e, ln_b    : [n_xi][n_modes] float32 (precision QS_FP32) or float64 (QS_FP64)
 *   n_modes >= 1, n_xi >= 1, half_window >= 0 (a window longer than the cells leaves no valid j)
 *   log_ratio     : [n_xi][n_modes] of the same type, or NULL
 *   first_e_cell  : int32 [n_modes], or NULL (at least one of the two outputs is required)
 * Ordered on hip_stream (NULL = null stream): one map kernel, with (for the staged forms,
 * when first_e_cell is given) a fill before it and a finish after it; no synchronization,
 * no allocation.  Calls
 * that write the same outputs concurrently on different streams race.
 * Errors: QS_ERR_ARG (sizes, precision, NULL inputs, both outputs NULL; nothing is launched),
 * QS_ERR_HIP (launch failure); qs_last_error() has the text.
 */
#ifndef QS_REGIME_H
#define QS_REGIME_H

#include <stddef.h>
#include <stdint.h>

#include "qs.h"

#ifdef __cplusplus
extern "C" {
#endif

qs_status qs_regime_map(const void *ln_e, const void *ln_b, int64_t n_modes, int32_t n_xi, int32_t half_window,
                        int32_t precision, void *log_ratio, int32_t *first_e_cell, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* QS_REGIME_H */
