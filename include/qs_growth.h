/*
 * Growth maps: answers to scattered queries of how much a mode has grown, from the solver
 * or from the learned surrogate (qs_mlp.h), with a held-out error table deciding which.
 *
 * A query is q = (ln n_b, ln gamma, k, xi, tau) for a single electron beam of density n_b
 * (in units of n_p) and Lorentz factor gamma, flat-top in xi, seeded with the uniform
 * extended disturbance S (Appendix C), inside the box
 *   n_b in [1e-3, 1e-1],  gamma in [10, 1e4],  k in [0.05, 4],  xi in [0, 200],
 *   tau in [0, tau_f],  tau_f = 10 sqrt(gamma / n_b)
 * (tau_f: ten e-folds of the temporal CFI rate sqrt(n_b/gamma) at large k, Eq. CFI_temporal).
 * Its answer is the growth of the windowed field amplitude over the seed,
 *   G = 1/2 ln( sum_i w_i A^2_(j-i) / sum_i w_i ) - ln S,   A^2 = |E|^2 + |B|^2,
 * at the cell j holding xi, with W = round(4 pi / h) cells (two plasma wavelengths, at least
 * one), Hann weights w_i = sin^2(pi (i + 1/2)/W) on the cells i = 0..min(j, W-1) behind and
 * at xi_j: the log amplitude smoothed over the two plasma wavelengths behind xi (A itself
 * carries the plasma-period ripple of the response; a one-wavelength box average leaves a
 * ripple wherever the envelope grows across the window, the Hann weights take it to second
 * order).  The solver's answer: the query's beam on cells of width h0 = 200/8192 (the finest
 * of the batched sweep, the same for every answer) reaching at least two cells beyond xi,
 * d_tau = tau_f/200, FP32 state, the windowed growth of every step's fields, bilinearly
 * interpolated between the two cell centres around xi and the two steps around tau.  A query sent to the solver must have finite values, gamma > 1, k >= 0, xi >= 0
 * and 0 <= tau <= 1e4 tau_f
 * (QS_ERR_ARG otherwise, naming the query).
 *
 * Box coordinates of a query (its place in the held-out error table), each in [-1, 1] inside
 * the box:  b = ( log10 n_b + 2, (log10 gamma - 2.5)/1.5, (k - 2.025)/1.975, xi/100 - 1,
 * 2 tau/tau_f - 1 ).
 * The surrogate's answer is B(q) + network(x(q)): the network (qs_mlp.h) learns the residual
 * over a closed-form baseline
 *   B = 1/2 ln(kappa^2 (1 + 3 k^2)/2) + J( M(ln cosh t, F), O ),
 *   F = 2 (sqrt(1 + t xi) - 1),  O = 3 ((1 + z)^(1/3) - 1),  z = (3 sqrt(3)/64) t_e^2 xi,
 *   t = Gamma_CFI tau = sqrt(n_b/gamma) k kappa^(1/2) tau,  kappa = 1/(1+k^2),
 *   t_e = t (1 + 1/(gamma k)^2)^(1/2),
 *   J(a, b) = ln(e^a + e^b - 1),  M(a, b) = -ln(e^-a + e^-b - e^-(a+b))
 * (the wavelength-averaged field of the extended disturbance at tau = 0, then the temporal
 * CFI growth of Appendix C held back near the front by F, whose exponent tends to the
 * spatiotemporal CFI one 2 sqrt(t xi) of Eq. CFI_ST, and overtaken deep in the beam by O,
 * whose exponent tends to the spatiotemporal OTSI one (3 sqrt(3)/4) t_e^(2/3) xi^(1/3) of
 * Eq. OTSI_ST, at the rate (Gamma_CFI^2 + beta^2)^(1/2) the longitudinal term gives it; for
 * a, b >= 0, J and M are 0 at a = b = 0, J(a, 0) = a, M(a, 0) = 0, and they tend to max and
 * min once both are large; F and O start linearly in t xi and z, so B is smooth in the
 * inputs and is the field level at tau = 0), from the inputs
 *   x = ( log10 n_b + 2, (log10(gamma k) - 2.1505)/2.4515, 2 log10(k/0.05)/log10(80) - 1,
 *         2 sqrt(xi/200) - 1, 2 sqrt(t/t_max) - 1 ),  t_max = 40/sqrt(17),
 * each in [-1, 1] inside the box (k floored at 1e-3 and xi, t at 0 so that any query has
 * finite inputs).  In these coordinates the continuum answer depends on n_b only through
 * the discretization: the master equation with tau -> Gamma_CFI tau keeps the one parameter
 * 1/(gamma k).
 *
 * Device arrays are float32 and caller-owned; calls are ordered on `hip_stream` (NULL =
 * null stream).  Errors: QS_ERR_ARG, QS_ERR_ALLOC, QS_ERR_HIP (qs_last_error has the text).
 */
#ifndef QS_GROWTH_H
#define QS_GROWTH_H

#include <stddef.h>
#include <stdint.h>

#include "qs.h"
#include "qs_mlp.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { QS_GROWTH_SURROGATE = 0, QS_GROWTH_SOLVER = 1, QS_GROWTH_AUTO = 2 };

/* Bins of the held-out error table: 8 per box coordinate, 8^5 in all, row-major in order. */
enum { QS_GROWTH_BINS = 32768 };

/* One solver instance whose snapshots feed qs_growth_targets / qs_growth_sample. */
typedef struct qs_growth_instance {
    double nb_over_np;   /* electron beam density n_b / n_p */
    double gamma_b;
    double length;       /* beam length L; cells of width h = L / n_xi */
    double d_tau;
    double seed_amp;     /* S of the uniform seed */
    int32_t n_xi;
    int32_t n_modes;
    const double *k;     /* host: |k| of each mode */
} qs_growth_instance;

/*
 * Training targets from solver snapshots (qs_step_tau layout, FP32): for every snapshot
 * t < n_snap, instance i, cell j and mode m, G[t][i][j][m] = the windowed growth above.
 * ln_e, ln_b, G: device [n_snap][sum_i n_xi_i n_modes_i] with instance i's block
 * [n_xi][n_modes] at the running offset.  inst: host array of n_inst descriptions.
 */
qs_status qs_growth_targets(const qs_growth_instance *inst, int32_t n_inst, const float *ln_e,
                            const float *ln_b, int32_t n_snap, float *G, void *hip_stream);

/*
 * Draw n training examples uniformly over all (snapshot, instance, cell, mode) entries of G
 * (entry number floor(u * total), u = top 53 bits of SplitMix64 output i of `seed`, over
 * 2^53).  snap_step: host [n_snap] step index of each snapshot (tau = step * d_tau).
 * Q: device [n][5] the entry's query (ln n_b, ln gamma, k, xi_j, tau) in float32;
 * T: device [n] its target G.
 */
qs_status qs_growth_sample(const qs_growth_instance *inst, int32_t n_inst, const float *G,
                           int32_t n_snap, const int32_t *snap_step, uint64_t seed, int64_t n,
                           float *Q, float *T, void *hip_stream);

/* The network inputs x (device [n][5], or NULL) and the baseline B (device [n], or NULL) of
 * queries q (device [n][5]); at least one output is required. */
qs_status qs_growth_features(const float *q, int64_t n, float *x, float *baseline, void *hip_stream);

/*
 * Held-out error table: per bin of the box coordinates, an upper estimate of the 99th
 * percentile of |B(q) + network(x(q)) - t| over the held-out examples in the bin: the upper
 * edge of the histogram bucket that holds it (so within a factor 2^(1/32) above the plain
 * percentile), buckets (1e-4 2^((b-1)/32), 1e-4 2^(b/32)] (b = 1..542; bucket 0 is [0, 1e-4],
 * bucket 543 everything above 1e-4 2^(542/32) ~ 12.5, reported as 3e38).  -1 where a bin holds
 * fewer than 32 examples.  Q, T: device held-out queries [n][5] and targets [n]; table: device
 * [QS_GROWTH_BINS].  Uses the network's stream; allocates 28 n bytes and a 71 MB histogram.
 */
qs_status qs_growth_calibrate(qs_mlp *net, const float *Q, const float *T, int64_t n, float *table);

/*
 * Answer n queries (device q [n][5]) into out (device [n]).
 *   QS_GROWTH_SURROGATE : B(q) + network(x(q)) for every query (net required).
 *   QS_GROWTH_SOLVER    : the solver for every query (net and table ignored; may be NULL).
 *   QS_GROWTH_AUTO      : the network where the query is inside the box and its bin's
 *                         held-out error is in [0, tol]; the solver elsewhere.
 * used_solver (device [n] bytes, optional): 1 where the solver answered.  AUTO picks out the
 * queries for the solver on the device and copies only those to the host.  The solver path
 * runs its queries as the modes of solver contexts, 32 queries of any beams per wavefront: in
 * units of each query's own step the model is the unit-density beam with the push
 * coefficients scaled by d_tau^2 (the same discrete solution).  Queries are sorted by the last
 * step they read and cut into chunks of at most 32768; a chunk's queries, sorted by the cells
 * they need, form instances of 32 that each reach two cells beyond their largest xi.  The
 * context marches without fields to the chunk's first step read, then writes the fields of
 * every later step, kept only for each instance's rear cells that the windows read, and the
 * answers are summed from those snapshots.  It allocates its buffers (within 16 GB per chunk)
 * and synchronizes.
 */
qs_status qs_growth_map(qs_mlp *net, const float *table, float tol, const float *q, int64_t n,
                        int32_t mode, float *out, uint8_t *used_solver, void *hip_stream);

/* Largest query count of one qs_growth_map_noalloc call (its scratch holds their inputs and
 * baselines). */
#define QS_GROWTH_NOALLOC_MAX 262144

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, hosts that forbid hipMalloc): qs_growth_map's network answers without any
 * allocation, synchronization or solver call.  For each of the n queries (device q [n][5]):
 *   out[i]          : the network's answer, bitwise equal to qs_growth_map in
 *                     QS_GROWTH_SURROGATE mode on the same network and queries;
 *   needs_solver[i] : 1 where QS_GROWTH_AUTO would send the query to the solver (outside the
 *                     box, no held-out estimate in its bin, or the estimate above tol, or
 *                     table == NULL), else 0; such answers are not to be trusted at tol and
 *                     the caller may pass those queries to qs_growth_map afterwards.
 * 0 <= n <= QS_GROWTH_NOALLOC_MAX (QS_ERR_ARG beyond, with nothing launched).  out, needs_solver:
 * device arrays of n elements; table: device [QS_GROWTH_BINS] or NULL.
 * Work is queued on the network's stream (qs_mlp_create), with no host synchronization.
 * The network inputs and baselines are staged in a fixed 6 MiB device array of the library (one per
 * device, held until the process ends, resolved on the first call on that device): calls
 * that overlap on one device, on any streams, race on it and must be serialized by the
 * caller.  The call after a parameter change also repacks the network's inference weights
 * (qs_mlp_forward), which is a kernel launch, not an allocation.
 * Errors: QS_ERR_ARG, QS_ERR_HIP (qs_last_error has the text).
 */
qs_status qs_growth_map_noalloc(qs_mlp *net, const float *table, float tol, const float *q, int64_t n, float *out,
                                uint8_t *needs_solver);

#ifdef __cplusplus
}
#endif

#endif /* QS_GROWTH_H */
