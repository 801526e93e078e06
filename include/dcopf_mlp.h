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

void dcopf_mlp_destroy(dcopf_mlp_t m);   /* NULL is a no-op                  */

#ifdef __cplusplus
}
#endif

#endif /* DCOPF_MLP_H */
