/*
 * dcopf_batch.h - batched projected dual ascent: many DCOPF instances (load
 * and cost scenarios) on one or more networks, advanced together.
 *
 * Every instance runs exactly the iteration of dcopf_dual.h (Section 3.3,
 * Algorithm 1 and its Adam / AdaGrad variants on the Lagrange dual of
 * Section 3; closed-form inner minimiser of Sections 3.1 / 3.2).  The paper
 * leaves solving many instances in parallel to future work (Sections 1 and
 * 5); here the instances of one network share its PTDF, so the two products
 * per iteration become dense GEMMs:
 *
 *     W^T = V^T P   (V = mu+ - mu-, [instances x lines] . [lines x columns])
 *     F^T = X^T P^T (X = injections at the generator buses)
 *
 * run on the matrix cores as split-BF16 products: each FP32 factor a is
 * written a_hi + a_lo with a_hi = bf16(a), a_lo = bf16(a - a_hi); the product
 * a b is formed as a_hi b_hi + a_hi b_lo + a_lo b_hi (optionally + a_lo b_lo)
 * with FP32 accumulation.  Line multipliers and velocities are FP32; lambda,
 * the reduced costs, the inner minimiser, the monitor gamma and the exact
 * bound are FP64.  The exact bound (dcopf_batch_bound) evaluates the dual
 * function with FP64 products (FP64 matrix cores).
 *
 * Errors, threading and stream semantics are those of dcopf_dual.h; the
 * message of a failed call is in dcopf_last_error().
 */
#ifndef DCOPF_BATCH_H
#define DCOPF_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include "dcopf_dual.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One network and the instances on it.  HOST pointers, copied at create.  */
typedef struct {
  int32_t n_bus, n_line, n_gen, slack;   /* as dcopf_problem                 */
  const double *H;        /* [n_line * n_bus] row-major PTDF, zero slack col */
  const int32_t *gen_bus; /* [n_gen]                                         */
  const double *p_min;    /* [n_gen] shared by the instances                 */
  const double *p_max;    /* [n_gen]                                         */
  const double *f_max;    /* [n_line] symmetric limits, > 0                  */
  int32_t n_inst;         /* instances on this network, >= 1; n_inst times
                             n_line (both padded) stays below 2^30           */
  const double *d;        /* [n_inst * n_bus] load of each instance          */
  const double *c;        /* [n_inst * n_gen] linear cost of each instance   */
  const double *q;        /* [n_inst * n_gen] quadratic cost (>= 0) or NULL  */
  double alpha, rho;      /* step size (> 0) and GDM momentum for this
                             network's instances                             */
} dcopf_batch_network;

typedef struct {
  int32_t rule;           /* DCOPF_RULE_GDM / ADAM / ADAGRAD                 */
  int32_t literal;        /* GDM reading, as dcopf_opts.literal              */
  double beta1, beta2, eps, decay;   /* as dcopf_opts                        */
  int32_t lolo;           /* 1: add the a_lo b_lo term (4 products)          */
  int32_t graph_iters;    /* iterations per captured HIP graph (0: direct)   */
  int32_t autotune;       /* 1: time the tile shapes at create and keep the
                             fastest per network; 0: built-in defaults       */
  int32_t gamma_cap;      /* monitor ring: last gamma_cap iterations are kept
                             (power of two, 1..65536)                        */
} dcopf_batch_opts;

typedef struct dcopf_batch_s *dcopf_batch_t;

/* Validates every network and instance like dcopf_dual_create (including
 * the per-instance balance check: DCOPF_E_INFEASIBLE names the instance),
 * uploads the PTDFs, builds the split-BF16 and FP64 panels, forms H d for
 * every instance in FP64, and sets the cold start (lambda = mu = 0).
 * Instance numbering is global: network 0's instances first.  Synchronises. */
dcopf_status dcopf_batch_create(const dcopf_batch_network *nets, int32_t n_nets,
                                const dcopf_batch_opts *opts, void *hip_stream,
                                dcopf_batch_t *out);

/* Enqueue n_iters >= 0 iterations of every instance.  Asynchronous.       */
dcopf_status dcopf_batch_step(dcopf_batch_t b, int64_t n_iters);

/* Exact FP64 dual value of every instance at its current iterate (valid
 * lower bounds, Remarks 1 and 2) into values[n_total]; the best value per
 * instance is tracked (dcopf_batch_best).  Synchronises.                    */
dcopf_status dcopf_batch_bound(dcopf_batch_t b, double *values);

/* Best exact bound per instance and the iteration it was evaluated at.     */
dcopf_status dcopf_batch_best(dcopf_batch_t b, double *values, int64_t *iters);

/* Iterate until every instance's best exact bound is within gap_tol of its
 * opt[i] (relative), or max_iters; bounds are evaluated every check_every
 * iterations.  first_hit[i] receives the iteration of the first bound within
 * the gap (-1 if never); may be NULL.  Synchronises.                       */
dcopf_status dcopf_batch_solve(dcopf_batch_t b, const double *opt, double gap_tol,
                               int64_t max_iters, int64_t check_every, int64_t *first_hit);

/* Monitor values gamma_k of iterations [first, first+count) for all
 * instances: out[(k - first) * n_total + i].  Synchronises.                */
dcopf_status dcopf_batch_gammas(dcopf_batch_t b, int64_t first, int64_t count, double *out);

/* Multipliers of network `net` (host doubles): lambda[n_inst],
 * mu_plus / mu_minus [n_inst * n_line].  get: any output may be NULL.
 * set (warm start): mu >= 0 and finite; this network's optimiser state is
 * reset to zero (other networks keep theirs) and the iteration counter of
 * the whole batch restarts at 0.  Synchronise.                             */
dcopf_status dcopf_batch_get_multipliers(dcopf_batch_t b, int32_t net, double *lambda,
                                         double *mu_plus, double *mu_minus);
dcopf_status dcopf_batch_set_multipliers(dcopf_batch_t b, int32_t net, const double *lambda,
                                         const double *mu_plus, const double *mu_minus);

/* Whole ascent state of network `net` (checkpoint / resume, or a start that
 * carries optimiser state; Section 3.3's rules keep a velocity or first
 * moment and a second moment per multiplier).  Host doubles, length
 * dcopf_batch_state_len(b, net) = 1 + 3 n_inst + 6 n_inst n_line:
 *   [0]                      iteration counter k (shared by every network of
 *                            the batch: it drives step decay and Adam's bias
 *                            correction)
 *   [1 .. 1+n_inst)          lambda per instance
 *   then n_inst each         lambda's velocity (GDM) or first moment (Adam),
 *                            lambda's second moment (Adam, AdaGrad)
 *   then n_inst x n_line     each of mu+, mu-, their velocities / first
 *                            moments, their second moments (instance-major)
 * The line state is stored in FP32: set_state rounds it to nearest.
 * set_state: mu and second moments >= 0, every value finite, k a
 * nonnegative integer, else DCOPF_E_INVALID (nothing changed); a length
 * other than state_len is DCOPF_E_STATE.  It sets the batch's counter to k
 * (the other networks keep their iterates and optimiser state) and restarts
 * this network's best bounds.  state_len returns 0 for a bad handle or
 * network.  Synchronise.                                                  */
size_t dcopf_batch_state_len(dcopf_batch_t b, int32_t net);
dcopf_status dcopf_batch_get_state(dcopf_batch_t b, int32_t net, double *buf, size_t len);
dcopf_status dcopf_batch_set_state(dcopf_batch_t b, int32_t net, const double *buf, size_t len);

/* The fallback of a learned warm start: `dst` runs its instances from a
 * predicted start, `src` the same instances (equal loads, instance by
 * instance, on a network of the same shape) from the cold start of
 * Algorithm 1, both for the same number of iterations.  Evaluates the exact
 * bound of every instance of both, and wherever the cold instance's bound
 * is larger, copies its whole state (multipliers, optimiser state, best
 * bound, primal sums) over the warm one on the device; `kept` (host, [n
 * instances], may be NULL) receives 1 there and 0 elsewhere.  `src` may
 * then be destroyed: `dst` continues with the better trajectory of every
 * instance.  DCOPF_E_STATE if the two are at different iterations,
 * DCOPF_E_INVALID for different shapes, loads or step rules.
 * Synchronises both streams.                                               */
dcopf_status dcopf_batch_adopt_better(dcopf_batch_t dst, int32_t dnet, dcopf_batch_t src,
                                      int32_t snet, int32_t *kept);

/* Primal recovery (an extension, as dcopf_dual_average / dcopf_dual_primal):
 * enable = 1 restarts the average of every instance's inner minimiser p*
 * over the following iterations (including those of time_phases, which
 * advance the batch); enable = 0 stops adding.  Synchronises.             */
dcopf_status dcopf_batch_average(dcopf_batch_t b, int32_t enable);

/* For network `net`: out[n_inst] receives each instance's averaged dispatch
 * cost, balance residual and line overloads (FP64 products on the device);
 * p_avg (host, [n_inst * n_gen], generator order) may be NULL.
 * DCOPF_E_STATE when no iteration has been averaged.  Synchronises.       */
dcopf_status dcopf_batch_primal(dcopf_batch_t b, int32_t net, dcopf_primal *out,
                                double *p_avg);

/* Repair (an extension, as dcopf_dual_repair) of every instance of network
 * `net`: the rounds of dcopf_dual_repair, with its constants, for all
 * instances at once (an instance stops at its own stop rule, overflow or
 * max_rounds).  p_in: host [n_inst * n_gen] in generator order, or NULL for
 * the current primal averages (DCOPF_E_STATE when none).  out[n_inst]
 * (dcopf_repair of dcopf_dual.h); p_out: host [n_inst * n_gen] or NULL.
 * Device buffers for the active rows (n_inst * 256 * (panel columns)
 * doubles) and the Gram matrices (n_inst * 256^2 doubles) are allocated by
 * the network's first repair and kept with the handle.  Synchronises.    */
dcopf_status dcopf_batch_repair(dcopf_batch_t b, int32_t net, const double *p_in,
                                int32_t max_rounds, dcopf_repair *out, double *p_out);

/* Start multipliers of every instance of network `net` from a DEVICE array
 * (FP32, row i = instance i, row stride ld >= 2 n_line + 1, laid out
 * [mu+ (n_line), mu- (n_line), lambda], as the warm-start network's output
 * of dcopf_mlp.h): mu is projected onto mu >= 0 on the device; the
 * optimiser state and best bounds restart as in set_multipliers.  For a
 * start computed on the GPU with no host round trip.  DCOPF_E_NONFINITE if
 * a value is not finite (the state is then unspecified).  Synchronises.  */
dcopf_status dcopf_batch_set_start_dev(dcopf_batch_t b, int32_t net, const float *Y,
                                       int32_t ld);

/* Tile shapes in use for network `net`: cfg[0], cfg[1] = instances x
 * columns of one W-product workgroup tile, cfg[2] = its K split (over
 * lines), cfg[3] = instances * 1000 + lines of one F-product tile.         */
dcopf_status dcopf_batch_info(dcopf_batch_t b, int32_t net, int32_t *cfg, int64_t *iters);

/* Pin the tile shapes of network `net` (cfg[0..3] encoded as in
 * dcopf_batch_info: tiles 128x64, 64x128 or 32x128; K split 1..32, clamped
 * to the K extent), e.g. to reuse an earlier autotuning result.  Results do
 * not depend on the tile shapes; the K split changes only the FP32
 * summation order.  Rebuilds the tile tables and the captured graph.
 * Synchronises.                                                            */
dcopf_status dcopf_batch_set_tiles(dcopf_batch_t b, int32_t net, const int32_t *cfg);

/* Measurement: run n_iters >= 1 real iterations (they advance the batch)
 * with events attached to each dispatch (start and end of that kernel
 * alone); ms_out[0..2] = average ms of the W product (with the lambda
 * step of the previous iteration), the unit pass (inner minimiser) and the
 * F product with the mu step.  Synchronises.                               */
dcopf_status dcopf_batch_time_phases(dcopf_batch_t b, int64_t n_iters, double *ms_out);

void dcopf_batch_destroy(dcopf_batch_t b);   /* NULL is a no-op              */

#ifdef __cplusplus
}
#endif

#endif /* DCOPF_BATCH_H */
