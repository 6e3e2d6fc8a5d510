/*
 * The growth-map surrogate as one library call: training from solver runs, and the file that
 * holds a trained network with its held-out error table (for qs_growth_map, qs_growth.h).
 *
 * Training (qs_surrogate_train), every step on the device:
 *   1. a training sweep of `train_instances` single-electron flat-top beams, n_b log-uniform
 *      in [1e-3, 1e-1], gamma log-uniform in [10, 1e4] (the pair (log10 n_b, log10 gamma)
 *      stratified: one uniform point in each cell of a near-square grid over the plane),
 *      length L uniform in [5, 200] in cells of the growth map's width h0 = 200/8192
 *      (N = round(L/h0) cells of a beam N h0 long), `modes` modes k uniform in
 *      [0.05, 4], `steps` steps of d_tau = tau_f/steps (tau_f = 10 sqrt(gamma/n_b)), FP32
 *      state, seeded with the uniform extended disturbance S = 1e-6 (Appendix C); snapshots
 *      at every one of the first `train_dense_steps` steps (where the growth starts fastest in
 *      the inputs), then every `train_snap_every` steps, and at the last step; the windowed
 *      growth G of every entry (qs_growth_targets) and `samples` examples drawn over all
 *      entries (qs_growth_sample), rounded down to whole batches;
 *   2. a held-out sweep with independent draws of `heldout_instances` beams (stratified the
 *      same way) of `heldout_modes` modes each, k_m = 0.05 + 3.95 (m + u)/heldout_modes with
 *      one uniform u per beam, every beam `heldout_length` long (so that xi is covered
 *      uniformly), snapshots every `heldout_snap_every` steps from an offset that runs through
 *      0 .. heldout_snap_every-1 with the chunk (below), so that held-out examples fall on
 *      every step, between the training snapshots as well as on them, and `heldout_samples`
 *      examples;
 *   3. the network (qs_mlp.h) trained on the residual G - B over the baseline B and the
 *      inputs x of qs_growth.h: initial weights uniform in +-1/sqrt(fan_in), the output
 *      layer scaled to the residuals' spread with its bias at their mean; AdamW (beta
 *      0.9/0.999, eps 1e-8, `weight_decay`) over contiguous batches of `batch` examples
 *      (a different batch order each epoch), `epochs` epochs, learning rate cosine-decayed
 *      from `lr` to `lr_min`;
 *   4. the held-out error table (qs_growth_calibrate) and statistics of the held-out errors
 *      |B + network - G|.
 * Draws come from SplitMix64 streams keyed by `seed`.  The sweeps run in chunks of
 * `chunk_instances` instances (the device memory of a chunk: its solver state and three
 * float32 arrays of (snapshots x cells x modes)).
 *
 * cfg_json: a flat JSON object of numbers overriding the defaults (NULL or "" = defaults):
 *   train_instances 256, heldout_instances 1024, modes 128, heldout_modes 32, steps 200,
 *   train_dense_steps 10, train_snap_every 5, heldout_snap_every 10, samples 1e7,
 *   heldout_samples 4e6,
 *   heldout_length 200, chunk_instances 64, epochs 60, batch 8192, lr 1e-3,
 *   lr_min 1e-5, weight_decay 0.01, seed 0.
 * out_path: file written (host path); stats: host array of QS_SURROGATE_STATS doubles or NULL:
 *   [0] held-out RMS error, [1] its 99th percentile, [2] its maximum, [3] the fraction of
 *   held-out examples within 1e-2, [4] the fraction of the error table's bins whose estimate
 *   is in [0, 1e-2], [5] the last batch's training loss, [6] seconds of data generation,
 *   [7] seconds of training.
 * The file: "QSSURR01", uint32 version 1, parameter count, bin count, metadata length;
 * float32 parameters (qs_mlp.h layout); float32 table [QS_GROWTH_BINS]; the metadata, a JSON
 * object of the configuration and the statistics (host byte order).
 * Work is ordered on hip_stream (NULL = null stream); the call allocates its device buffers
 * (about 48 bytes per training example plus 24 per held-out example, plus one chunk's sweep)
 * and synchronizes.  Errors: QS_ERR_ARG (configuration, file), QS_ERR_ALLOC, QS_ERR_HIP, and
 * any error of the solver calls it makes.
 */
#ifndef QS_SURROGATE_H
#define QS_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "qs.h"
#include "qs_growth.h"
#include "qs_mlp.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { QS_SURROGATE_STATS = 8 };

typedef struct qs_surrogate qs_surrogate;

qs_status qs_surrogate_train(const char *cfg_json, const char *out_path, void *hip_stream, double *stats);

/*
 * Load a file written by qs_surrogate_train on the current device: a network (its stream is
 * hip_stream) and the device copy of its error table, owned by the returned handle.
 * Errors: QS_ERR_ARG (missing file, not a surrogate file of this library), QS_ERR_ALLOC,
 * QS_ERR_HIP.
 */
qs_status qs_surrogate_load(const char *path, void *hip_stream, qs_surrogate **out);

/* The loaded network and table (device [QS_GROWTH_BINS]) to pass to qs_growth_map /
 * qs_growth_map_noalloc; owned by the handle (NULL for a NULL handle). */
qs_mlp *qs_surrogate_net(const qs_surrogate *s);
const float *qs_surrogate_table(const qs_surrogate *s);

/* Release the network and the table.  NULL is ignored. */
void qs_surrogate_free(qs_surrogate *s);

#ifdef __cplusplus
}
#endif

#endif /* QS_SURROGATE_H */
