/*
 * dcopf_mlp.h - the learned warm start: a dense network that maps the load
 * vector of an instance to initial multipliers (mu+, mu-, lambda) for the
 * dual ascent, which otherwise starts from lambda = mu = 0 (Section 3.3,
 * Algorithm 1).  This part is not in the paper; any reported bound is still
 * an exact dual value (Remarks 1 and 2 hold for every mu >= 0), so a poor
 * prediction costs iterations, never validity.
 *
 * Network: n_in -> h1 -> h2 -> n_out, GELU (erf form) after each hidden
 * layer, linear output.  Weights are kept as FP32 masters and used as BF16
 * copies (both orientations) in the matrix-core products, FP32 accumulation;
 * training minimises the mean squared error of a batch with Adam (bias
 * corrected).  Weight layout: W_l is [out x in] row-major, b_l is [out].
 *
 * Data pointers of forward / train_step are DEVICE pointers on the handle's
 * stream; get/set_params use HOST buffers.  Errors as in dcopf_dual.h.
 */
#ifndef DCOPF_MLP_H
#define DCOPF_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "dcopf_dual.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_in, h1, h2, n_out;  /* layer widths, each in [1, 65536]          */
  int32_t max_batch;            /* largest batch of forward / train_step     */
  double beta1, beta2, eps;     /* Adam                                      */
} dcopf_mlp_config;

typedef struct dcopf_mlp_s *dcopf_mlp_t;

/* Allocate the network; parameters start at zero (use set_params).         */
dcopf_status dcopf_mlp_create(const dcopf_mlp_config *cfg, void *hip_stream,
                              dcopf_mlp_t *out);

/* Parameter count and host transfer: params = [W1, b1, W2, b2, W3, b3]
 * concatenated (FP32).  set_params also resets the Adam moments and step.  */
size_t dcopf_mlp_param_count(dcopf_mlp_t m);
dcopf_status dcopf_mlp_get_params(dcopf_mlp_t m, float *params, size_t len);
dcopf_status dcopf_mlp_set_params(dcopf_mlp_t m, const float *params, size_t len);

/* Forward pass: X [batch x n_in] FP32 (device) -> Y [batch x n_out] FP32
 * (device).  Asynchronous.                                                 */
dcopf_status dcopf_mlp_forward(dcopf_mlp_t m, const float *X, int32_t batch, float *Y);

/* One training step on a batch: forward, mean squared error against
 * T [batch x n_out] (device FP32), backward, Adam with step size lr.  If
 * loss is not NULL it receives the batch loss before the step (host,
 * synchronises); otherwise asynchronous.                                   */
dcopf_status dcopf_mlp_train_step(dcopf_mlp_t m, const float *X, const float *T,
                                  int32_t batch, double lr, double *loss);

/* Gradients of the last train_step (before the Adam update), host FP32,
 * same layout as params; for checking against a reference.  Synchronises. */
dcopf_status dcopf_mlp_get_grads(dcopf_mlp_t m, float *grads, size_t len);

/* Measurement: average ms of one train_step over n >= 1 steps on a fixed
 * batch (HIP events).  Parameters are restored afterwards.                */
dcopf_status dcopf_mlp_time_train(dcopf_mlp_t m, const float *X, const float *T,
                                  int32_t batch, int32_t n, double *ms);

/* Standardisation of the data the network learns from (a scaling of each
 * input and each target, so that every column has mean 0 and spread 1):
 *
 * column_stats: per column of A [rows x cols] (device FP32, row-major) its
 *   mean and standard deviation (population form, FP64 sums), written to
 *   mean[cols] and std[cols] (device FP32); a deviation of at most
 *   1e-12 (|mean| + 1) becomes 1 (a constant column is left unscaled).
 * standardize: out = (A - mean) / std per column (inverse = 0), or
 *   out = A * std + mean (inverse = 1); A, out [rows x cols] device FP32
 *   (out may equal A).
 * fold_standardizers: the parameters become those of the same network
 *   acting on raw inputs and returning raw outputs, for a network trained
 *   on standardised ones: W1 / std_x (per input column), b1 - W1 (mean_x /
 *   std_x), std_y W3 (per output row), std_y b3 + mean_y; FP64 sums.  The
 *   Adam moments are reset (the network is then for inference).  Device
 *   FP32 vectors x_mean, x_std [n_in], y_mean, y_std [n_out].
 *
 * All asynchronous on the handle's stream; DCOPF_E_INVALID for NULL
 * pointers or sizes out of range.                                          */
dcopf_status dcopf_mlp_column_stats(dcopf_mlp_t m, const float *A, int32_t rows, int32_t cols,
                                    float *mean, float *std);
dcopf_status dcopf_mlp_standardize(dcopf_mlp_t m, const float *A, int32_t rows, int32_t cols,
                                   const float *mean, const float *std, int32_t inverse,
                                   float *out);
dcopf_status dcopf_mlp_fold_standardizers(dcopf_mlp_t m, const float *x_mean,
                                          const float *x_std, const float *y_mean,
                                          const float *y_std);

void dcopf_mlp_destroy(dcopf_mlp_t m);   /* NULL is a no-op                  */

#ifdef __cplusplus
}
#endif

#endif /* DCOPF_MLP_H */
