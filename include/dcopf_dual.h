/*
 * dcopf_dual.h - C ABI of the MI355X projected dual-ascent DCOPF library.
 *
 * The method (arXiv 2406.13191, "GPU-Accelerated DCOPF using Gradient-Based
 * Optimization"): DC optimal power flow (Section 2, eq. DCOPF)
 *
 *     min_p  sum_g c_g p_g + q_g p_g^2
 *     s.t.   1^T p = 1^T d                              (power balance)
 *            -f_max <= H (C_g p - d) <= f_max           (PTDF line limits)
 *            p_min <= p <= p_max                        (generator box)
 *
 * is solved through its Lagrange dual (Section 3, eqs. lagrangian, dual
 * function, dual).  For multipliers lambda (balance, free) and mu+, mu- >= 0
 * (the two sides of every line limit), the inner minimisation over the box
 * has a closed form (Section 3.1 dual norm, eq. LP dual; Section 3.2, eq.
 * QP_finalgamma maximised over s): every generator sits at p_min / p_max by
 * the sign of its reduced cost r_g = c_g - lambda + (H^T (mu+ - mu-))[bus g]
 * (linear cost; the midpoint when r_g == 0) or at clip(-r_g / (2 q_g))
 * (quadratic cost).  The dual value
 *
 *     G = sum_g (r_g p*_g + q_g p*_g^2) + lambda 1^T d
 *         - (mu+ - mu-)^T H d - (mu+ + mu-)^T f_max
 *
 * is a valid lower bound on the optimal cost for any lambda and mu >= 0
 * (Remarks 1 and 2).  Its supergradient is the constraint residual at p*:
 * d/dlambda = 1^T d - 1^T p*, d/dmu+- = +-H (C_g p* - d) - f_max.  The ascent
 * (Section 3.3, Algorithm 1 and its Adam / AdaGrad variants) steps along it
 * and projects mu onto mu >= 0.
 *
 * Sign convention: lambda here is the marginal price (the canonical form's
 * A = -1^T), so the reduced cost is c - lambda 1 + C_g^T H^T (mu+ - mu-).
 *
 * All functions return a dcopf_status; on failure dcopf_last_error() gives a
 * message (thread-local, valid until the next call on that thread).  No call
 * throws across the ABI.  Handles are not thread-safe: use one handle from
 * one thread at a time.  Device work is enqueued on the HIP stream given at
 * create (NULL = the null stream); calls documented as "synchronises" wait
 * for that stream.
 */
#ifndef DCOPF_DUAL_H
#define DCOPF_DUAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DCOPF_OK = 0,
  DCOPF_E_INVALID = -1,     /* bad argument; nothing was changed */
  DCOPF_E_NOMEM = -2,       /* device or host allocation failed */
  DCOPF_E_HIP = -3,         /* a HIP runtime call failed */
  DCOPF_E_NONFINITE = -4,   /* a NaN/Inf appeared in the iterate or bound */
  DCOPF_E_INFEASIBLE = -5,  /* the instance is certified infeasible */
  DCOPF_E_STATE = -7        /* state buffer of the wrong length */
} dcopf_status;

/* Device memory of the handles.  Every buffer a handle owns (panels, state,
 * workspaces, the temporaries of its calls) comes from the allocator that
 * was installed on the creating thread when the handle was created, and
 * goes back to it when the handle is destroyed (or, for a temporary, when
 * its call returns).  Without one, hipMalloc and hipFree serve.  A caller
 * that manages device memory itself (PyTorch's caching allocator, a pool)
 * installs its pair here, so the library allocates nothing on its own:
 *
 *   alloc(bytes, stream, ctx): device memory of at least `bytes` bytes,
 *     256-byte aligned, usable on the current device by work on `stream`
 *     (the handle's stream); NULL when it cannot (the call then returns
 *     DCOPF_E_NOMEM);
 *   free(ptr, bytes, stream, ctx): returns a block alloc gave, after the
 *     work enqueued on `stream` that uses it (the release is stream
 *     ordered: the library does not wait before it).
 *
 * dcopf_set_allocator(NULL, NULL, NULL) restores hipMalloc / hipFree; one
 * of the two functions alone is DCOPF_E_INVALID.  The setting is per host
 * thread and applies to handles (and dcopf_ptdf calls) made after it; each
 * handle keeps the pair it was created with.                              */
typedef void *(*dcopf_alloc_fn)(size_t bytes, void *hip_stream, void *ctx);
typedef void (*dcopf_free_fn)(void *ptr, size_t bytes, void *hip_stream, void *ctx);
dcopf_status dcopf_set_allocator(dcopf_alloc_fn alloc, dcopf_free_fn free, void *ctx);

/* One DCOPF instance in the paper's statement (Section 2, eq. DCOPF).
 * All pointers are HOST memory; they are read during dcopf_dual_create and
 * may be freed by the caller when it returns.                              */
typedef struct {
  int32_t n_bus;            /* buses, >= 2                                   */
  int32_t n_line;           /* lines, >= 1                                   */
  int32_t n_gen;            /* generators, >= 1                              */
  int32_t slack;            /* slack bus index; column `slack` of H is zero  */
  const double *H;          /* [n_line * n_bus] row-major PTDF H_a (Section 2:
                               H = Omega E (E^T Omega E)^{-1} with a zero
                               slack column)                                 */
  const int32_t *gen_bus;   /* [n_gen] bus of each generator (C_g as a map)  */
  const double *c;          /* [n_gen] linear cost, $/MWh                    */
  const double *q;          /* [n_gen] quadratic cost $/MW^2h (>= 0); NULL =
                               all zero (the LP of Section 3.1)              */
  const double *p_min;      /* [n_gen] MW                                    */
  const double *p_max;      /* [n_gen] MW, p_min <= p_max                    */
  const double *d;          /* [n_bus] load, MW                              */
  const double *f_max;      /* [n_line] symmetric line limit, MW, > 0        */
} dcopf_problem;

enum { DCOPF_RULE_GDM = 0, DCOPF_RULE_ADAM = 1, DCOPF_RULE_ADAGRAD = 2 };
enum { DCOPF_PREC_FP64 = 0, DCOPF_PREC_FP32 = 1 };
enum { DCOPF_PANEL_GENBUS = 0, DCOPF_PANEL_ALLBUS = 1 };

/* Ascent options (Section 3.3).                                            */
typedef struct {
  int32_t rule;        /* DCOPF_RULE_*: gradient with momentum (Algorithm 1),
                          Adam, AdaGrad                                     */
  int32_t literal;     /* GDM only: 1 also applies Algorithm 1's separately
                          listed gradient update theta += alpha grad after
                          the velocity update; 0 = heavy-ball (velocity only) */
  double alpha;        /* step size, > 0                                     */
  double rho;          /* GDM momentum in [0, 1)                             */
  double beta1, beta2; /* Adam moment decays in [0, 1)                       */
  double eps;          /* Adam / AdaGrad denominator guard, > 0              */
  double decay;        /* step decay: alpha_k = alpha / (1 + decay k), >= 0  */
  int32_t precision;   /* DCOPF_PREC_FP64: every product in FP64.
                          DCOPF_PREC_FP32: the two PTDF products per iteration
                          in FP32 (FP32 accumulation); reduced costs, inner
                          minimiser, residual subtraction, updates, lambda and
                          the monitor gamma in FP64; dcopf_dual_bound always
                          evaluates in FP64.                                */
  int32_t panel;       /* DCOPF_PANEL_GENBUS: the products use only the H
                          columns of buses that host a generator (the others
                          multiply zero injections).  DCOPF_PANEL_ALLBUS: the
                          full H in both products (literal bus-vector form).
                          Both give the same dual values.                   */
  int32_t graph_iters; /* iterations per captured HIP graph; 0 = direct
                          launches                                          */
  int32_t qp_dual;     /* DCOPF_QP_CLOSED (0): a quadratic unit's inner
                          minimiser is the clip of -r / 2q, the exact maximum
                          over the paper's auxiliary s.  DCOPF_QP_ITERATED (1):
                          the paper's QP dual as printed (Section 3.2, eq.
                          QP_finalgamma): every unit keeps its own s, the
                          unit is bang-bang on r + 2 q m - sqrt(q) s (m the
                          centre of its box), and s takes the same GDM step
                          as lambda and mu along -sqrt(q)(p* - m) - s/2.  An
                          ablation: requires rule GDM, literal 0, decay 0;
                          get_state, set_state and time_phases then return
                          DCOPF_E_INVALID; the monitor gamma is the value of
                          that dual, dcopf_dual_bound the exact (closed-form)
                          dual at the same lambda and mu.                  */
  int32_t scheme;      /* how an iteration reads the panel (same arithmetic
                          up to FP32 summation order; results bitwise
                          reproducible either way):
                          DCOPF_SCHEME_TWO_PASS: a column pass over P^T
                          (w = P^T v, units, x) then a line pass over P
                          (F = P x, step and projection): the panel is read
                          twice, with two launches and little beyond it.
                          DCOPF_SCHEME_READ_ONCE: the line pass also forms,
                          from the same rows of P, the per-workgroup
                          partials of the next w = P^T v (Algorithm 1's two
                          products from one read), and a unit pass sums them
                          per column: the panel is read once, plus the
                          partials (workgroups x columns).  Rows wider than
                          16 chunks per lane of a workgroup (FP32 panels of
                          more than 16,384 columns, FP64 of 8,192) only have
                          the two-pass scheme (DCOPF_E_INVALID if asked).
                          DCOPF_SCHEME_AUTO (0): read-once for panels of at
                          least 10 MiB in the loop precision, two-pass below
                          (launch latency, not bytes, bounds those).       */
} dcopf_opts;

enum { DCOPF_QP_CLOSED = 0, DCOPF_QP_ITERATED = 1 };
enum { DCOPF_SCHEME_AUTO = 0, DCOPF_SCHEME_TWO_PASS = 1, DCOPF_SCHEME_READ_ONCE = 2 };

typedef struct dcopf_dual_s *dcopf_dual_t;

/* Build the solver: validates the instance and options, uploads H, gathers
 * the panel (FP32 and/or FP64, both orientations), forms H d in FP64, and
 * sets the cold start lambda = mu = 0 and zero optimiser state (Algorithm 1
 * initialisation).  `hip_stream` is a hipStream_t (NULL = null stream).
 * Errors: DCOPF_E_INVALID (dimensions, indices, non-finite values, p_min >
 * p_max, q < 0, f_max <= 0, nonzero slack column, bad options),
 * DCOPF_E_INFEASIBLE (sum p_min > 1^T d or sum p_max < 1^T d),
 * DCOPF_E_NOMEM, DCOPF_E_HIP.  On error *out is set to NULL. Synchronises. */
dcopf_status dcopf_dual_create(const dcopf_problem *prob, const dcopf_opts *opts,
                               void *hip_stream, dcopf_dual_t *out);

/* Enqueue n_iters >= 0 ascent iterations (Algorithm 1 loop body: reduced
 * costs, inner minimiser, residuals, step + projection; gamma_k of each
 * iterate recorded).  Asynchronous.                                        */
dcopf_status dcopf_dual_step(dcopf_dual_t h, int64_t n_iters);

/* Exact FP64 dual value G at the current iterate (all products FP64); a
 * valid lower bound on the optimal cost (Remarks 1 and 2).  The best value
 * seen by this call is tracked (dcopf_dual_best).  Optional outputs (may be
 * NULL): lambda (1), mu_plus / mu_minus ([n_line], host).  Synchronises.
 * DCOPF_E_NONFINITE if the value or iterate is not finite.                  */
dcopf_status dcopf_dual_bound(dcopf_dual_t h, double *value, double *lambda,
                              double *mu_plus, double *mu_minus);

/* Best exact bound recorded by dcopf_dual_bound / dcopf_dual_solve and the
 * iteration at which it was evaluated (-inf / -1 if none yet).             */
dcopf_status dcopf_dual_best(dcopf_dual_t h, double *value, int64_t *iteration);

typedef struct {
  double bound;          /* best exact FP64 lower bound                      */
  double gamma_last;     /* monitor gamma of the last iterate                */
  double gap;            /* (opt - bound) / |opt|, NaN when opt is NaN       */
  int64_t iters;         /* iterations done by this handle in total          */
  int64_t iter_of_bound; /* iteration at which `bound` was evaluated         */
  int32_t status;        /* 1 gap reached, 2 |d gamma| < tol (Algorithm 1's
                            stopping test), 3 max_iters, 0 otherwise          */
} dcopf_result;

/* Run the ascent until the exact bound is within gap_tol of `opt`
 * (relative; ignored when opt is NaN), or |gamma_k - gamma_{k-1}| <
 * dgamma_tol (ignored when <= 0), or max_iters more iterations; the exact
 * bound is evaluated every `check_every` (>= 1) iterations and at the end.
 * Returns DCOPF_E_INFEASIBLE when a bound exceeds the largest possible cost
 * sum_g max_p (c_g p + q_g p^2) (the dual is then unbounded).  Synchronises. */
dcopf_status dcopf_dual_solve(dcopf_dual_t h, double opt, double gap_tol,
                              double dgamma_tol, int64_t max_iters,
                              int64_t check_every, dcopf_result *out);

/* Monitor values gamma_k (dual value at iterate k, from the products of the
 * chosen precision) for iterations [first, first + count) of this handle;
 * only the last 2^20 iterations are kept.  Synchronises.                   */
dcopf_status dcopf_dual_gammas(dcopf_dual_t h, int64_t first, int64_t count,
                               double *out);

/* State (host doubles, length dcopf_dual_state_len): [iteration, lambda,
 * lambda velocity / first moment, lambda second moment, 0, mu+ [n_line],
 * mu- [n_line], velocity or first moment of mu+ and mu- [2 n_line], second
 * moment of mu+ and mu- [2 n_line]].  set_state is a warm start or resume;
 * mu must be >= 0 and finite (DCOPF_E_INVALID otherwise).  Synchronise.    */
size_t dcopf_dual_state_len(dcopf_dual_t h);
dcopf_status dcopf_dual_get_state(dcopf_dual_t h, double *buf, size_t len);
dcopf_status dcopf_dual_set_state(dcopf_dual_t h, const double *buf, size_t len);

/* Measurement: n_iters >= 1 real iterations from the current iterate (column
 * pass and line pass alternating as in dcopf_dual_step), each launch with
 * start/stop events attached to its dispatch (the kernel's own timestamps);
 * ms_out[0], ms_out[1] receive the average ms of the column pass (w = P^T v
 * and the inner minimiser) and of the line pass (F = P x - f_d and the mu
 * step).  The iterate and iteration count are restored.  Synchronises.     */
dcopf_status dcopf_dual_time_phases(dcopf_dual_t h, int64_t n_iters, double *ms_out);

/* Primal recovery (an extension; the paper reports only lower bounds and
 * takes optima from a solver).  The ergodic average pbar of the inner
 * minimisers p*_k over a window of iterations is a primal candidate: the
 * constraints are affine, so its residuals are the averaged supergradients,
 * which vanish as the window grows, and its cost then approaches the optimum
 * from above the lower bound.                                               */
typedef struct {
  double cost;          /* sum_g c_g pbar_g + q_g pbar_g^2                   */
  double balance;       /* 1^T d - 1^T pbar (MW)                             */
  double max_overload;  /* largest (F_l - f_max,l)_+ or (-F_l - f_max,l)_+
                           over lines, F = H (C_g pbar - d) (MW)             */
  double sum_overload;  /* sum of those overloads over lines and directions */
  int64_t iterations;   /* iterations averaged                               */
  int32_t n_overloaded; /* line directions with a positive overload          */
} dcopf_primal;

/* enable = 1: restart the average; every following iteration adds its p*.
 * enable = 0: stop adding (the sum is kept for dcopf_dual_primal).  The
 * iterations of dcopf_dual_time_phases never add.  Synchronises.          */
dcopf_status dcopf_dual_average(dcopf_dual_t h, int32_t enable);

/* pbar = (sum of p*) / iterations and its cost and residuals, evaluated in
 * FP64 on the device.  p_avg (host, [n_gen], generator order) may be NULL.
 * DCOPF_E_STATE when no iteration has been averaged.  Synchronises.       */
dcopf_status dcopf_dual_primal(dcopf_dual_t h, dcopf_primal *out, double *p_avg);

/* Repair (an extension, as the primal average): a feasible dispatch near a
 * primal candidate.  Its cost is an upper bound on the optimum, so with the
 * exact lower bound it certifies the gap without an external solver.
 * Starting from p = the candidate clipped to the generator box, each round
 * evaluates F = H (C_g p - d) and 1^T d - 1^T p in FP64; stops when no line
 * direction is violated and |1^T d - 1^T p| <= 1e-9 max(1, 1^T d);
 * otherwise adds every violated line direction to an active set (in line
 * order; a line held in one direction switches if the other is violated;
 * at most 255 lines) and moves p by the correction of least
 * sum_g dp_g^2 / w_g, w_g = max(min(p_g - p_min_g, p_max_g - p_g),
 * 1e-3 (p_max_g - p_min_g)), that holds every active line 1e-6 MW inside
 * its limit and closes the balance (Gram system with a ridge of 1e-12 of
 * its largest diagonal, Cholesky in FP64), then clips p to the box.       */
typedef struct {
  double cost;          /* sum_g c_g p_g + q_g p_g^2 of the result: an upper
                           bound on the optimum when feasible                */
  double balance;       /* 1^T d - 1^T p (MW)                                */
  double max_overload;  /* largest line overload of the result (MW)         */
  double max_shift;     /* largest |p_g - candidate_g| after the first clip  */
  int32_t feasible;     /* 1: the stop rule was met                          */
  int32_t rounds;       /* correction steps taken                            */
  int32_t n_active;     /* line limits held                                  */
  int32_t pad;
} dcopf_repair;

/* p_in: host [n_gen] in generator order, or NULL for the current primal
 * average (DCOPF_E_STATE when nothing has been averaged).  max_rounds >= 0.
 * p_out: host [n_gen], generator order, may be NULL.  A candidate the rounds
 * do not repair is not an error: feasible = 0.  DCOPF_E_INVALID for a
 * negative max_rounds or a non-finite p_in.  Synchronises.                */
dcopf_status dcopf_dual_repair(dcopf_dual_t h, const double *p_in, int32_t max_rounds,
                               dcopf_repair *out, double *p_out);

/* Panel width (number of H columns the products use) and iterations done. */
dcopf_status dcopf_dual_info(dcopf_dual_t h, int32_t *n_cols, int64_t *iters);

/* The iteration scheme the handle runs (DCOPF_SCHEME_TWO_PASS or
 * DCOPF_SCHEME_READ_ONCE, resolved from DCOPF_SCHEME_AUTO at create) and,
 * for read-once, the number of line-pass workgroups, each of which writes
 * one partial of P^T v per iteration (0 for two-pass).  Either output may
 * be NULL.                                                                 */
dcopf_status dcopf_dual_scheme(dcopf_dual_t h, int32_t *scheme, int32_t *line_groups);

/* Free all device and host memory of the handle.  NULL is a no-op.        */
void dcopf_dual_destroy(dcopf_dual_t h);

/* Message of the last failed call on this thread ("" if none).           */
const char *dcopf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DCOPF_DUAL_H */
