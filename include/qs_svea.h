/*
 * Envelope-approximation (SVEA) variant of the spectral path, to run beside the full model.
 *
 * Sec. III.B of the paper writes the transverse master equation without its gamma^-2 term,
 * [(d_xi^2 + 1) d_tau^2 - Gamma^2] n_p = delta(xi) delta(tau), substitutes n_p = N e^{-i xi}
 * and, under the slowly varying envelope approximation (d_xi N << N), keeps
 *     d_tau^2 d_xi N = (i/2) Gamma^2 N + (i/2) delta(xi) delta(tau),
 * the equation of the earlier spatiotemporal OTSI theory, which the paper shows to fail near
 * the beam front (where spatiotemporal CFI dominates) and to share the leading exponential
 * of the full model far behind it.  This library solves, per transverse mode,
 *     d_tau^2 d_xi n = a n + delta(xi) delta(tau)        (N = (i/2) n for a = (i/2) Gamma^2)
 * as the first-order system  d_tau n = m,  d_tau m = a * integral_0^xi n dxi', started after
 * the impulse from n = 0, m = 1 behind the front.  Cells j = 0 .. n_xi - 1 of width h hold
 * n_j, m_j (cell values); the integral at a cell centre is h sum_{i<j} n_i + (h/2) n_j; classic
 * fourth-order Runge-Kutta in tau with all four stages in one causal sweep down the cells
 * (stage s at cell j needs only stage s-1 through cell j), FP64 throughout.  The state of
 * a mode is rescaled by a power of two (exactly) whenever its largest component leaves
 * [2^-100, 2^100]; log2_scale[mode] accumulates the exponents, so the true state is
 * state * 2^log2_scale.
 *
 * Layouts (all device memory, caller-owned): n and m are complex FP64, interleaved
 * (re, im), in blocks of 64 modes: the value of (cell j, mode k) is element
 * ((k / 64) n_xi + j) 64 + k % 64, so a buffer holds ceil(n_modes / 64) 64 n_xi complex
 * values (padding entries are written by the seed and otherwise ignored); a is complex FP64
 * [n_modes]; log2_scale is int32 [n_modes].  Calls are ordered on hip_stream (NULL = null stream) and
 * do not synchronize.  Errors: QS_ERR_ARG (sizes, NULL pointers; nothing is launched),
 * QS_ERR_HIP (launch failure); qs_last_error() has the text.
 */
#ifndef QS_SVEA_H
#define QS_SVEA_H

#include <stddef.h>
#include <stdint.h>

#include "qs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Host helper: a[mode] = (i/2) Gamma_CFI(k_mode)^2 with Gamma_CFI^2 = sum_s q_s^2 n_bs / (m_s
 * gamma) * k^2 / (1 + k^2) (Eq. CFI_temporal), for n_modes wavenumbers k (host arrays; a is
 * complex, interleaved).  Errors: QS_ERR_ARG. */
qs_status qs_svea_coefficients(int32_t n_species, const double *q, const double *m, const double *nb_over_np,
                               double gamma_b, int64_t n_modes, const double *k, double *a);

/* State right after the impulse: n = 0, m = 1 in every cell, log2_scale = 0. */
qs_status qs_svea_seed_impulse(int64_t n_modes, int32_t n_xi, double *n, double *m, int32_t *log2_scale,
                               void *hip_stream);

/* Advance every mode by n_steps steps of d_tau (n_steps >= 0; one launch; modes are
 * independent).  h > 0 is the cell width, a the per-mode coefficient (typically
 * (i/2) Gamma_CFI(k)^2, Eq. CFI_temporal). */
qs_status qs_svea_step(int64_t n_modes, int32_t n_xi, double h, const double *a, double d_tau, int32_t n_steps,
                       double *n, double *m, int32_t *log2_scale, void *hip_stream);

/* ln |N| = ln |n| - ln 2 + log2_scale ln 2 per (cell, mode) into ln_abs [n_xi][n_modes]
 * (FP64): the envelope of the paper's normalization (N = (i/2) n); -inf where n = 0. */
qs_status qs_svea_ln_envelope(int64_t n_modes, int32_t n_xi, const double *n, const int32_t *log2_scale,
                              double *ln_abs, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* QS_SVEA_H */
