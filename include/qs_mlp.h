/*
 * Growth-map surrogate network of libqs: a 5 -> 512 -> 512 -> 512 -> 512 -> 1 multilayer
 * perceptron with the exact GELU activation x * Phi(x) (Hendrycks and Gimpel, 2016),
 * trained by mean squared error with AdamW (Loshchilov and Hutter, 2019), for fast queries
 * of the log growth of a mode, ln A(n_b, gamma, k, xi, tau), learned from solver runs.
 * (The paper motivates the quasistatic model by the cost of full simulations; the
 * surrogate answers scattered growth queries without marching.)
 *
 * Arithmetic: the three 512 x 512 products run on the matrix cores with bfloat16 operands
 * (round to nearest even from float32) and float32 accumulation; the first layer (5
 * inputs) and the last (1 output), the bias additions, the activation and all reductions
 * are float32.  Stored activations h1..h4 are bfloat16.  Master weights and the AdamW
 * moments are float32.  Training evaluates Phi with the float32 error function; inference
 * (qs_mlp_forward) reads Phi from a table of cubic Hermite pieces (16 per unit on [-6, 6],
 * interpolation error below 3e-8), so the two forward passes agree to float32 rounding
 * except where an activation lands on a bfloat16 rounding boundary.
 *
 * Parameter layout (float32, host arrays of qs_mlp_param_count() elements), in order:
 *   W1 [512][5], b1 [512], W2 [512][512], b2 [512], W3 [512][512], b3 [512],
 *   W4 [512][512], b4 [512], W5 [1][512], b5 [1]
 * (W_l[out][in]; layer l computes z = W_l h + b_l).
 *
 * All device pointers below are caller-owned device memory; host pointers are marked.
 * Calls are ordered on the stream given at creation and do not synchronize unless stated.
 * Errors are returned as qs_status (see qs.h); qs_last_error() gives the text.
 */
#ifndef QS_MLP_H
#define QS_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "qs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qs_mlp qs_mlp;

/* Number of float32 parameters (and gradients) in the layout above. */
int64_t qs_mlp_param_count(void);

/*
 * Create a network with zero parameters on the current device.  max_batch (a positive
 * multiple of 128, at most 2^20) bounds the rows of one training step; the library
 * allocates its activation, gradient and optimizer buffers for it (about
 * 5.5 KB x max_batch + 13 MB).  hip_stream: the stream every call is ordered on (NULL =
 * the null stream).  Errors: QS_ERR_ARG, QS_ERR_ALLOC.
 */
qs_status qs_mlp_create(int32_t max_batch, void *hip_stream, qs_mlp **out);

/* Replace / read the float32 master parameters (host arrays, layout above; synchronizes).
 * Setting the parameters also clears the AdamW moments and its step counter. */
qs_status qs_mlp_set_params(qs_mlp *net, const float *host_params);
qs_status qs_mlp_get_params(qs_mlp *net, float *host_params);

/*
 * Inference: y[i] = network(x[i]) for i < n (n >= 0, any size, independent of max_batch).
 * x: device float32 [n][5]; y: device float32 [n].  One persistent kernel per 2^25 queries
 * keeps every activation on chip; it uses no buffer of the network besides its parameters.
 * The first call after the parameters change (qs_mlp_set_params, qs_mlp_adamw) first
 * repacks the inference copy of W2..W4 (one small kernel on the same stream).
 */
qs_status qs_mlp_forward(qs_mlp *net, const float *x, int64_t n, float *y);

/*
 * Gradients of the mean squared error L = (1/batch) sum_i (network(x_i) - t_i)^2 with
 * respect to all parameters, kept inside the network (layout above).  x: device float32
 * [batch][5]; t: device float32 [batch]; batch a positive multiple of 128 <= max_batch.
 * loss (host, optional): receives L (synchronizes when given).
 */
qs_status qs_mlp_grads(qs_mlp *net, const float *x, const float *t, int32_t batch, double *loss);

/* Copy the gradients of the last qs_mlp_grads call to a host array, or replace them from
 * one (e.g. gradients computed elsewhere, before qs_mlp_adamw); both synchronize. */
qs_status qs_mlp_get_grads(qs_mlp *net, float *host_grads);
qs_status qs_mlp_set_grads(qs_mlp *net, const float *host_grads);

/*
 * One AdamW step with the current gradients, for every parameter w (weights and biases):
 *   m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
 *   w <- w - lr ( m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps) + weight_decay w ),  t = step count.
 */
qs_status qs_mlp_adamw(qs_mlp *net, double lr, double beta1, double beta2, double eps, double weight_decay);

/* qs_mlp_grads followed by qs_mlp_adamw (beta1 0.9, beta2 0.999, eps 1e-8, weight decay 0.01). */
qs_status qs_mlp_train_step(qs_mlp *net, const float *x, const float *t, int32_t batch, double lr,
                            double *loss);

/* Release the network and its buffers.  NULL is ignored. */
void qs_mlp_free(qs_mlp *net);

/*
 * Test hook, host only (no device call): build the arguments of every matrix-core GEMM of one
 * training step on `batch` rows of a network created with `max_batch`, at the buffer offsets
 * a real network uses, and check them against what the GEMM kernel assumes (whole 128 x 128
 * output tiles and 64-long reduction chunks, 16-byte aligned rows long enough for every
 * split, a grid inside the device limits, every epilogue output present); qs_mlp_grads makes
 * the same check before each launch.  Returns 0 when all hold, 1 otherwise, -1 for batch
 * sizes the network would refuse; msg (host, msg_len bytes, may be NULL) gets the split count
 * or what failed.
 */
int32_t qs_debug_mlp_gemm_check(int32_t max_batch, int32_t batch, char *msg, int32_t msg_len);

#ifdef __cplusplus
}
#endif

#endif /* QS_MLP_H */
