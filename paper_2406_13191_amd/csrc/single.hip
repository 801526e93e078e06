// Single-instance projected dual ascent for DCOPF on CDNA4 (gfx950).
//
// One ascent iteration (Section 3.3, Algorithm 1) is two streaming passes
// over the generator-bus panel P = H[:, U] of the PTDF (U = the buses that
// host a generator; Section 2 eq. DCOPF, the injections of all other buses
// are the constant loads, folded into f_d = H d once):
//
//   column pass  (rows of P^T, coalesced):  w = P^T v  with v = mu+ - mu-,
//                then per generator the reduced cost r = c - lambda + w[col],
//                the closed-form inner minimiser p* (Section 3.1 dual norm /
//                Section 3.2 clipped quadratic), phi = r p* + q p*^2 and the
//                per-column injection x = sum of p* at that bus.  The last
//                workgroup reduces sum p* and sum phi (fixed order) and takes
//                the lambda step with the balance residual 1^T d - 1^T p*.
//   line pass    (rows of P, coalesced):  F = P x - f_d, the residuals
//                +-F - f_max, the step and projection mu <- max(0, .) per
//                line, and the next v.  The last workgroup finishes the dual
//                value gamma_k = sum phi + lambda 1^T d - v^T f_d
//                - (mu+ + mu-)^T f_max of the iterate the pass started from.
//
// Both passes keep their vector (v or x) in LDS and stream the panel with
// 16-byte loads, one wavefront per row, wave-shuffle reductions.  Cross-
// workgroup sums use per-workgroup partials reduced by the last workgroup in
// index order, so results are bitwise reproducible.
#include "common.h"
#include "../../include/dcopf_dual.h"

#include <cmath>
#include <cstring>
#include <limits>
#include <vector>
#include <algorithm>
#include <numeric>

namespace dcopf {

thread_local std::string g_err;
void set_error(const std::string &m) { g_err = m; }
const char *get_error() { return g_err.c_str(); }

// Scalars shared by the kernels of one handle (device memory).
struct DevScalars {
  double lam, v_lam, s_lam;   // balance multiplier and its optimiser state
  double psum, gamma_gen;     // column pass: sum p*, sum phi + lambda D
  double alpha_k, c1, c2;     // step size of this iteration, Adam corrections
  double gamma_last;          // monitor value of the last finished iterate
  double D;                   // 1^T d
  double bound_gen, bound_value;
  long long k;                // iterations done
  long long pad;
};

struct StepParams {
  int rule, literal;
  double alpha, rho, beta1, beta2, eps, decay;
};

// Inner minimiser of r p + q p^2 over [lo, hi] (Section 3.1 / 3.2).
__device__ __forceinline__ double inner_min(double r, double q, double lo, double hi) {
  if (q > 0.0) return fmin(fmax(-r / (2.0 * q), lo), hi);
  if (r > 0.0) return lo;
  if (r < 0.0) return hi;
  return 0.5 * (lo + hi);
}

// Dot product of one row (length ld, multiple of 64 elements, 16-byte
// aligned) with a vector, by one wavefront.  Two independent accumulators
// keep two 16-byte loads in flight per lane.
template <typename T>
__device__ __forceinline__ T row_dot(const T *__restrict__ row, const T *__restrict__ x,
                                     int ld, int lane) {
  using V = typename Vec16<T>::type;
  constexpr int NV = Vec16<T>::n;
  const V *r = reinterpret_cast<const V *>(row);
  const V *xv = reinterpret_cast<const V *>(x);
  const int nv = ld / NV;
  T a0 = 0, a1 = 0;
  int i = lane;
  for (; i + kWave < nv; i += 2 * kWave) {
    V p0 = __builtin_nontemporal_load(r + i);
    V p1 = __builtin_nontemporal_load(r + i + kWave);
    a0 = fma_vec(p0, xv[i], a0);
    a1 = fma_vec(p1, xv[i + kWave], a1);
  }
  if (i < nv) a0 = fma_vec(__builtin_nontemporal_load(r + i), xv[i], a0);
  return wave_sum(a0 + a1);
}

// ---------------------------------------------------------------------------
// Column pass.  ITER: part of an ascent iteration (updates lambda); otherwise
// the exact-bound evaluation (writes bound_gen only).  STAGE: vector in LDS.
// ---------------------------------------------------------------------------
template <typename T, bool ITER, bool STAGE>
__global__ __launch_bounds__(256) void colpass_kernel(
    const T *__restrict__ PT, int n_cols, int ldl, const T *__restrict__ vvec,
    const int *__restrict__ seg, const int *__restrict__ gperm,
    const double *__restrict__ c, const double *__restrict__ q,
    const double *__restrict__ pmin, const double *__restrict__ pmax,
    DevScalars *sc, T *__restrict__ x_out, double *__restrict__ part,
    unsigned *counter, StepParams prm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  __shared__ bool last_flag;
  const T *vs = vvec;
  if (STAGE) {
    T *vl = reinterpret_cast<T *>(smem_raw);
    using V = typename Vec16<T>::type;
    constexpr int NV = Vec16<T>::n;
    for (int i = threadIdx.x; i < ldl / NV; i += blockDim.x)
      reinterpret_cast<V *>(vl)[i] = reinterpret_cast<const V *>(vvec)[i];
    __syncthreads();
    vs = vl;
  }
  const double lam = sc->lam;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  double psum = 0.0, phisum = 0.0;
  for (int j = blockIdx.x * nw + wave; j < n_cols; j += gridDim.x * nw) {
    T w = row_dot<T>(PT + (size_t)j * ldl, vs, ldl, lane);
    if (lane == 0) {
      const double wd = (double)w;
      double xj = 0.0;
      for (int k = seg[j]; k < seg[j + 1]; ++k) {
        const int g = gperm[k];
        const double r = c[g] - lam + wd;
        const double p = inner_min(r, q[g], pmin[g], pmax[g]);
        phisum += r * p + q[g] * p * p;
        psum += p;
        xj += p;
      }
      if (ITER) x_out[j] = (T)xj;
    }
  }
  const double bp = block_sum(psum, red);
  const double bphi = block_sum(phisum, red);
  if (threadIdx.x == 0) {
    store_agent(part + 2 * blockIdx.x, bp);
    store_agent(part + 2 * blockIdx.x + 1, bphi);
  }
  if (!last_block_done(counter, &last_flag)) return;
  double tp = 0.0, tphi = 0.0;
  for (int b = threadIdx.x; b < gridDim.x; b += blockDim.x) {
    tp += load_agent(part + 2 * b);
    tphi += load_agent(part + 2 * b + 1);
  }
  tp = block_sum(tp, red);
  tphi = block_sum(tphi, red);
  if (threadIdx.x != 0) return;
  const double D = sc->D;
  if (!ITER) {
    sc->bound_gen = tphi + lam * D;
    return;
  }
  sc->psum = tp;
  sc->gamma_gen = tphi + lam * D;
  // step size and Adam bias corrections of this iteration
  const double kk = (double)sc->k;
  const double a = prm.alpha / (1.0 + prm.decay * kk);
  const double c1 = 1.0 - pow(prm.beta1, kk + 1.0);
  const double c2 = 1.0 - pow(prm.beta2, kk + 1.0);
  sc->alpha_k = a;
  sc->c1 = c1;
  sc->c2 = c2;
  const double g = D - tp;  // balance residual: supergradient in lambda
  double lamn = lam;
  if (prm.rule == DCOPF_RULE_GDM) {
    const double v = prm.rho * sc->v_lam + a * g;
    sc->v_lam = v;
    lamn = lam + v;
    if (prm.literal) lamn += a * g;
  } else if (prm.rule == DCOPF_RULE_ADAM) {
    const double m = prm.beta1 * sc->v_lam + (1.0 - prm.beta1) * g;
    const double s = prm.beta2 * sc->s_lam + (1.0 - prm.beta2) * g * g;
    sc->v_lam = m;
    sc->s_lam = s;
    lamn = lam + a * (m / c1) / (sqrt(s / c2) + prm.eps);
  } else {
    const double s = sc->s_lam + g * g;
    sc->s_lam = s;
    lamn = lam + a * g / (sqrt(s) + prm.eps);
  }
  sc->lam = lamn;
}

// ---------------------------------------------------------------------------
// Line pass: F = P x - f_d, residuals, mu step + projection, next v.
// ---------------------------------------------------------------------------
template <typename T, bool STAGE>
__global__ __launch_bounds__(256) void linepass_kernel(
    const T *__restrict__ P, int n_lines, int ldc, const T *__restrict__ x_in,
    const double *__restrict__ fd, const double *__restrict__ flim,
    double *__restrict__ mu_p, double *__restrict__ mu_m, double *__restrict__ v_p,
    double *__restrict__ v_m, double *__restrict__ s_p, double *__restrict__ s_m,
    T *__restrict__ v_out, DevScalars *sc, double *__restrict__ part, unsigned *counter,
    StepParams prm, double *__restrict__ gam_buf, long long gam_mask) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  __shared__ bool last_flag;
  const T *xs = x_in;
  if (STAGE) {
    T *xl = reinterpret_cast<T *>(smem_raw);
    using V = typename Vec16<T>::type;
    constexpr int NV = Vec16<T>::n;
    for (int i = threadIdx.x; i < ldc / NV; i += blockDim.x)
      reinterpret_cast<V *>(xl)[i] = reinterpret_cast<const V *>(x_in)[i];
    __syncthreads();
    xs = xl;
  }
  const double a = sc->alpha_k, c1 = sc->c1, c2 = sc->c2;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  double lsum = 0.0;
  for (int l = blockIdx.x * nw + wave; l < n_lines; l += gridDim.x * nw) {
    T f = row_dot<T>(P + (size_t)l * ldc, xs, ldc, lane);
    if (lane == 0) {
      const double F = (double)f - fd[l];
      const double gp = F - flim[l], gm = -F - flim[l];
      const double mp = mu_p[l], mm = mu_m[l];
      lsum += (mp - mm) * fd[l] + (mp + mm) * flim[l];
      double np_, nm_;
      if (prm.rule == DCOPF_RULE_GDM) {
        const double vp = prm.rho * v_p[l] + a * gp;
        const double vm = prm.rho * v_m[l] + a * gm;
        v_p[l] = vp;
        v_m[l] = vm;
        np_ = mp + vp;
        nm_ = mm + vm;
        if (prm.literal) {
          np_ += a * gp;
          nm_ += a * gm;
        }
      } else if (prm.rule == DCOPF_RULE_ADAM) {
        const double m1 = prm.beta1 * v_p[l] + (1.0 - prm.beta1) * gp;
        const double m2 = prm.beta1 * v_m[l] + (1.0 - prm.beta1) * gm;
        const double s1 = prm.beta2 * s_p[l] + (1.0 - prm.beta2) * gp * gp;
        const double s2 = prm.beta2 * s_m[l] + (1.0 - prm.beta2) * gm * gm;
        v_p[l] = m1;
        v_m[l] = m2;
        s_p[l] = s1;
        s_m[l] = s2;
        np_ = mp + a * (m1 / c1) / (sqrt(s1 / c2) + prm.eps);
        nm_ = mm + a * (m2 / c1) / (sqrt(s2 / c2) + prm.eps);
      } else {
        const double s1 = s_p[l] + gp * gp, s2 = s_m[l] + gm * gm;
        s_p[l] = s1;
        s_m[l] = s2;
        np_ = mp + a * gp / (sqrt(s1) + prm.eps);
        nm_ = mm + a * gm / (sqrt(s2) + prm.eps);
      }
      np_ = fmax(np_, 0.0);
      nm_ = fmax(nm_, 0.0);
      mu_p[l] = np_;
      mu_m[l] = nm_;
      v_out[l] = (T)(np_ - nm_);
    }
  }
  const double bl = block_sum(lsum, red);
  if (threadIdx.x == 0) store_agent(part + blockIdx.x, bl);
  if (!last_block_done(counter, &last_flag)) return;
  double t = 0.0;
  for (int b = threadIdx.x; b < gridDim.x; b += blockDim.x) t += load_agent(part + b);
  t = block_sum(t, red);
  if (threadIdx.x == 0) {
    const double gam = sc->gamma_gen - t;
    const long long k = sc->k;
    gam_buf[k & gam_mask] = gam;
    sc->gamma_last = gam;
    sc->k = k + 1;
  }
}

// Line terms of the exact bound: sum_l (mu+ - mu-) f_d + (mu+ + mu-) f_max.
__global__ __launch_bounds__(256) void bound_lines_kernel(
    const double *__restrict__ mu_p, const double *__restrict__ mu_m,
    const double *__restrict__ fd, const double *__restrict__ flim, int n_lines,
    DevScalars *sc, double *__restrict__ part, unsigned *counter) {
  __shared__ double red[4];
  __shared__ bool last_flag;
  double s = 0.0;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n_lines;
       l += gridDim.x * blockDim.x)
    s += (mu_p[l] - mu_m[l]) * fd[l] + (mu_p[l] + mu_m[l]) * flim[l];
  s = block_sum(s, red);
  if (threadIdx.x == 0) store_agent(part + blockIdx.x, s);
  if (!last_block_done(counter, &last_flag)) return;
  double t = 0.0;
  for (int b = threadIdx.x; b < gridDim.x; b += blockDim.x) t += load_agent(part + b);
  t = block_sum(t, red);
  if (threadIdx.x == 0) sc->bound_value = sc->bound_gen - t;
}

// v = mu+ - mu- in T, zero padded to ld.
template <typename T>
__global__ void make_v_kernel(const double *mu_p, const double *mu_m, int n, int ld, T *v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ld; i += gridDim.x * blockDim.x)
    v[i] = i < n ? (T)(mu_p[i] - mu_m[i]) : (T)0;
}

// ---- setup (once per handle) ----------------------------------------------
// Panel gather: out[l, j] = H[l, cols[j]] (line-major, zero padded to ldc).
template <typename T>
__global__ void gather_kernel(const double *__restrict__ H, int n_bus, int n_lines,
                              const int *__restrict__ cols, int n_cols, int ldc,
                              T *__restrict__ out) {
  const int l = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ldc; j += gridDim.x * blockDim.x)
    out[(size_t)l * ldc + j] = j < n_cols ? (T)H[(size_t)l * n_bus + cols[j]] : (T)0;
}

// Transpose through an LDS tile: outT[j, l] = in[l, j] (zero padded to ldl).
template <typename T>
__global__ void transpose_kernel(const T *__restrict__ in, int n_lines, int ldc, int n_cols,
                                 int ldl, T *__restrict__ outT) {
  __shared__ T tile[32][33];
  const int j0 = blockIdx.x * 32, l0 = blockIdx.y * 32;
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int l = l0 + r, j = j0 + threadIdx.x;
    tile[r][threadIdx.x] = (l < n_lines && j < ldc) ? in[(size_t)l * ldc + j] : (T)0;
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int j = j0 + r, l = l0 + threadIdx.x;
    if (j < n_cols && l < ldl) outT[(size_t)j * ldl + l] = tile[threadIdx.x][r];
  }
}

// f_d = H d in FP64 over the full PTDF (one wavefront per line).
__global__ __launch_bounds__(256) void hd_kernel(const double *__restrict__ H, int n_bus,
                                                 int n_lines, const double *__restrict__ d,
                                                 double *__restrict__ fd) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int l = blockIdx.x * nw + wave; l < n_lines; l += gridDim.x * nw) {
    double s = 0.0;
    for (int b = lane; b < n_bus; b += kWave) s = fma(H[(size_t)l * n_bus + b], d[b], s);
    s = wave_sum(s);
    if (lane == 0) fd[l] = s;
  }
}

}  // namespace dcopf

// ===========================================================================
// Host side
// ===========================================================================
using namespace dcopf;

namespace {

constexpr long long kGamCap = 1LL << 20;  // monitor ring capacity (power of 2)

template <typename T> T *dalloc(size_t n, dcopf_status *st) {
  void *p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
    *st = DCOPF_E_NOMEM;
    return nullptr;
  }
  return static_cast<T *>(p);
}

bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

struct dcopf_dual_s {
  int n_bus = 0, n_lines = 0, n_gen = 0, n_cols = 0, ldc = 0, ldl = 0;
  dcopf_opts opts{};
  StepParams prm{};
  hipStream_t stream = nullptr;
  // panels
  float *P32 = nullptr, *P32T = nullptr;
  double *P64 = nullptr, *P64T = nullptr;
  // data
  double *fd = nullptr, *fmax = nullptr, *c = nullptr, *q = nullptr, *pmin = nullptr,
         *pmax = nullptr;
  int *seg = nullptr, *gperm = nullptr;
  // state
  double *mu_p = nullptr, *mu_m = nullptr, *v_p = nullptr, *v_m = nullptr, *s_p = nullptr,
         *s_m = nullptr;
  void *vbuf = nullptr, *xbuf = nullptr;  // loop precision vectors (padded)
  double *v64b = nullptr;                 // FP64 v for the exact bound
  double *part_a = nullptr, *part_b = nullptr, *part_c = nullptr;
  unsigned *counters = nullptr;
  DevScalars *sc = nullptr;
  double *gam = nullptr;
  // launch shapes
  int grid_col = 0, grid_line = 0, grid_bnd_col = 0, grid_bnd_line = 0;
  size_t lds_col = 0, lds_line = 0, lds_bnd = 0;
  bool stage_col = false, stage_line = false, stage_bnd = false;
  // graph of graph_iters iterations
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // host bookkeeping
  long long iters = 0;
  double best = -INFINITY;
  long long best_iter = -1;
  double cost_ub = INFINITY;  // largest possible generation cost
};

namespace {

template <typename T>
void launch_colpass(dcopf_dual_s *h, hipStream_t s) {
  T *PT = std::is_same<T, float>::value ? (T *)h->P32T : (T *)h->P64T;
  T *v = (T *)h->vbuf, *x = (T *)h->xbuf;
  if (h->stage_col)
    colpass_kernel<T, true, true><<<h->grid_col, 256, h->lds_col, s>>>(
        PT, h->n_cols, h->ldl, v, h->seg, h->gperm, h->c, h->q, h->pmin, h->pmax, h->sc, x,
        h->part_a, h->counters + 0, h->prm);
  else
    colpass_kernel<T, true, false><<<h->grid_col, 256, 0, s>>>(
        PT, h->n_cols, h->ldl, v, h->seg, h->gperm, h->c, h->q, h->pmin, h->pmax, h->sc, x,
        h->part_a, h->counters + 0, h->prm);
}

template <typename T>
void launch_linepass(dcopf_dual_s *h, hipStream_t s) {
  T *P = std::is_same<T, float>::value ? (T *)h->P32 : (T *)h->P64;
  T *v = (T *)h->vbuf, *x = (T *)h->xbuf;
  if (h->stage_line)
    linepass_kernel<T, true><<<h->grid_line, 256, h->lds_line, s>>>(
        P, h->n_lines, h->ldc, x, h->fd, h->fmax, h->mu_p, h->mu_m, h->v_p, h->v_m, h->s_p,
        h->s_m, v, h->sc, h->part_b, h->counters + 1, h->prm, h->gam, kGamCap - 1);
  else
    linepass_kernel<T, false><<<h->grid_line, 256, 0, s>>>(
        P, h->n_lines, h->ldc, x, h->fd, h->fmax, h->mu_p, h->mu_m, h->v_p, h->v_m, h->s_p,
        h->s_m, v, h->sc, h->part_b, h->counters + 1, h->prm, h->gam, kGamCap - 1);
}

void launch_phase(dcopf_dual_s *h, hipStream_t s, int phase) {
  const bool fp32 = h->opts.precision == DCOPF_PREC_FP32;
  if (phase == 0) {
    if (fp32) launch_colpass<float>(h, s); else launch_colpass<double>(h, s);
  } else {
    if (fp32) launch_linepass<float>(h, s); else launch_linepass<double>(h, s);
  }
}

void launch_iters(dcopf_dual_s *h, hipStream_t s, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    launch_phase(h, s, 0);
    launch_phase(h, s, 1);
  }
}

void refresh_v(dcopf_dual_s *h) {
  const int blocks = (int)std::min<int64_t>(1024, (h->ldl + 255) / 256);
  if (h->opts.precision == DCOPF_PREC_FP32)
    make_v_kernel<float><<<blocks, 256, 0, h->stream>>>(h->mu_p, h->mu_m, h->n_lines, h->ldl,
                                                         (float *)h->vbuf);
  else
    make_v_kernel<double><<<blocks, 256, 0, h->stream>>>(h->mu_p, h->mu_m, h->n_lines,
                                                          h->ldl, (double *)h->vbuf);
}

dcopf_status validate(const dcopf_problem *p, const dcopf_opts *o) {
  if (!p || !o) return set_error("null problem or options"), DCOPF_E_INVALID;
  if (p->n_bus < 2 || p->n_line < 1 || p->n_gen < 1)
    return set_error("need n_bus >= 2, n_line >= 1, n_gen >= 1"), DCOPF_E_INVALID;
  if (p->slack < 0 || p->slack >= p->n_bus)
    return set_error("slack bus out of range"), DCOPF_E_INVALID;
  if (!p->H || !p->gen_bus || !p->c || !p->p_min || !p->p_max || !p->d || !p->f_max)
    return set_error("null data pointer"), DCOPF_E_INVALID;
  const size_t nl = p->n_line, nb = p->n_bus, ng = p->n_gen;
  if ((double)nl * (double)nb > 4.0e9)
    return set_error("H larger than 4e9 entries"), DCOPF_E_INVALID;
  for (size_t g = 0; g < ng; ++g)
    if (p->gen_bus[g] < 0 || p->gen_bus[g] >= p->n_bus)
      return set_error("gen_bus[" + std::to_string(g) + "] out of range"), DCOPF_E_INVALID;
  if (!finite_all(p->H, nl * nb)) return set_error("H has non-finite entries"), DCOPF_E_INVALID;
  if (!finite_all(p->c, ng) || !finite_all(p->p_min, ng) || !finite_all(p->p_max, ng) ||
      !finite_all(p->d, nb) || !finite_all(p->f_max, nl) || (p->q && !finite_all(p->q, ng)))
    return set_error("non-finite problem data"), DCOPF_E_INVALID;
  for (size_t g = 0; g < ng; ++g) {
    if (p->p_min[g] > p->p_max[g])
      return set_error("p_min > p_max at generator " + std::to_string(g)), DCOPF_E_INVALID;
    if (p->q && p->q[g] < 0.0)
      return set_error("q < 0 at generator " + std::to_string(g)), DCOPF_E_INVALID;
  }
  for (size_t l = 0; l < nl; ++l)
    if (!(p->f_max[l] > 0.0))
      return set_error("f_max <= 0 at line " + std::to_string(l)), DCOPF_E_INVALID;
  for (size_t l = 0; l < nl; ++l)
    if (p->H[l * nb + p->slack] != 0.0)
      return set_error("H column of the slack bus is not zero"), DCOPF_E_INVALID;
  if (!(o->alpha > 0.0) || !std::isfinite(o->alpha))
    return set_error("alpha must be > 0"), DCOPF_E_INVALID;
  if (o->rule < 0 || o->rule > 2) return set_error("unknown rule"), DCOPF_E_INVALID;
  if (!(o->rho >= 0.0 && o->rho < 1.0)) return set_error("rho must be in [0,1)"), DCOPF_E_INVALID;
  if (o->rule == DCOPF_RULE_ADAM &&
      !(o->beta1 >= 0.0 && o->beta1 < 1.0 && o->beta2 >= 0.0 && o->beta2 < 1.0))
    return set_error("beta1, beta2 must be in [0,1)"), DCOPF_E_INVALID;
  if (o->rule != DCOPF_RULE_GDM && !(o->eps > 0.0))
    return set_error("eps must be > 0"), DCOPF_E_INVALID;
  if (!(o->decay >= 0.0) || !std::isfinite(o->decay))
    return set_error("decay must be >= 0"), DCOPF_E_INVALID;
  if (o->precision != DCOPF_PREC_FP64 && o->precision != DCOPF_PREC_FP32)
    return set_error("unknown precision"), DCOPF_E_INVALID;
  if (o->panel != DCOPF_PANEL_GENBUS && o->panel != DCOPF_PANEL_ALLBUS)
    return set_error("unknown panel mode"), DCOPF_E_INVALID;
  if (o->graph_iters < 0 || o->graph_iters > 4096)
    return set_error("graph_iters must be in [0, 4096]"), DCOPF_E_INVALID;
  double smin = 0, smax = 0, D = 0;
  for (size_t g = 0; g < ng; ++g) smin += p->p_min[g], smax += p->p_max[g];
  for (size_t b = 0; b < nb; ++b) D += p->d[b];
  if (D < smin - 1e-9 * std::max(1.0, std::fabs(D)) ||
      D > smax + 1e-9 * std::max(1.0, std::fabs(D)))
    return set_error("total load outside [sum p_min, sum p_max]"), DCOPF_E_INFEASIBLE;
  return DCOPF_OK;
}

void free_handle(dcopf_dual_s *h) {
  if (!h) return;
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  void *ptrs[] = {h->P32, h->P32T, h->P64, h->P64T, h->fd, h->fmax, h->c, h->q,
                  h->pmin, h->pmax, h->seg, h->gperm, h->mu_p, h->mu_m, h->v_p, h->v_m,
                  h->s_p, h->s_m, h->vbuf, h->xbuf, h->v64b, h->part_a, h->part_b,
                  h->part_c, h->counters, h->sc, h->gam};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete h;
}

int grid_for(int rows, int rows_per_block, int max_blocks) {
  int g = (rows + rows_per_block - 1) / rows_per_block;
  return std::max(1, std::min(g, max_blocks));
}

}  // namespace

extern "C" {

const char *dcopf_last_error(void) { return get_error(); }

dcopf_status dcopf_dual_create(const dcopf_problem *p, const dcopf_opts *o, void *hip_stream,
                               dcopf_dual_t *out) {
  if (!out) return set_error("out is NULL"), DCOPF_E_INVALID;
  *out = nullptr;
  set_error("");
  dcopf_status st = validate(p, o);
  if (st != DCOPF_OK) return st;
  auto *h = new dcopf_dual_s();
  h->stream = (hipStream_t)hip_stream;
  h->opts = *o;
  h->prm = StepParams{o->rule, o->literal, o->alpha, o->rho, o->beta1, o->beta2, o->eps,
                      o->decay};
  h->n_bus = p->n_bus;
  h->n_lines = p->n_line;
  h->n_gen = p->n_gen;
  const int nb = p->n_bus, nl = p->n_line, ng = p->n_gen;
  // panel columns: distinct generator buses (sorted) or all buses
  std::vector<int> cols;
  if (o->panel == DCOPF_PANEL_ALLBUS) {
    cols.resize(nb);
    std::iota(cols.begin(), cols.end(), 0);
  } else {
    cols.assign(p->gen_bus, p->gen_bus + ng);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  }
  const int nc = (int)cols.size();
  std::vector<int> col_of_bus(nb, -1);
  for (int j = 0; j < nc; ++j) col_of_bus[cols[j]] = j;
  std::vector<int> gperm(ng);
  std::iota(gperm.begin(), gperm.end(), 0);
  std::stable_sort(gperm.begin(), gperm.end(), [&](int a, int b) {
    return col_of_bus[p->gen_bus[a]] < col_of_bus[p->gen_bus[b]];
  });
  std::vector<int> seg(nc + 1, 0);
  for (int g = 0; g < ng; ++g) seg[col_of_bus[p->gen_bus[g]] + 1]++;
  for (int j = 0; j < nc; ++j) seg[j + 1] += seg[j];
  h->n_cols = nc;
  h->ldc = (int)round_up(nc, 64);
  h->ldl = (int)round_up(nl, 64);
  const bool fp32 = o->precision == DCOPF_PREC_FP32;
  const size_t esz = fp32 ? 4 : 8;

  // launch shapes: 4 wavefronts per workgroup
  h->grid_col = grid_for(nc, 4, 4096);
  h->grid_line = grid_for(nl, 8, 4096);
  h->grid_bnd_col = grid_for(nc, 4, 4096);
  h->grid_bnd_line = grid_for(nl, 256, 1024);
  h->lds_col = (size_t)h->ldl * esz;
  h->lds_line = (size_t)h->ldc * esz;
  h->lds_bnd = (size_t)h->ldl * 8;
  h->stage_col = h->lds_col <= 64 * 1024;
  h->stage_line = h->lds_line <= 64 * 1024;
  h->stage_bnd = h->lds_bnd <= 64 * 1024;

  st = DCOPF_OK;
  const size_t panel = (size_t)nl * h->ldc, panelT = (size_t)nc * h->ldl;
  if (fp32) {
    h->P32 = dalloc<float>(panel, &st);
    h->P32T = dalloc<float>(panelT, &st);
  } else {
    h->P64 = dalloc<double>(panel, &st);
  }
  h->P64T = dalloc<double>(panelT, &st);
  h->fd = dalloc<double>(nl, &st);
  h->fmax = dalloc<double>(nl, &st);
  h->c = dalloc<double>(ng, &st);
  h->q = dalloc<double>(ng, &st);
  h->pmin = dalloc<double>(ng, &st);
  h->pmax = dalloc<double>(ng, &st);
  h->seg = dalloc<int>(nc + 1, &st);
  h->gperm = dalloc<int>(ng, &st);
  double **state[] = {&h->mu_p, &h->mu_m, &h->v_p, &h->v_m, &h->s_p, &h->s_m};
  for (double **s : state) *s = dalloc<double>(nl, &st);
  h->vbuf = dalloc<unsigned char>((size_t)h->ldl * esz, &st);
  h->xbuf = dalloc<unsigned char>((size_t)h->ldc * esz, &st);
  h->v64b = dalloc<double>(h->ldl, &st);
  h->part_a = dalloc<double>(2 * (size_t)std::max(h->grid_col, h->grid_bnd_col), &st);
  h->part_b = dalloc<double>((size_t)h->grid_line, &st);
  h->part_c = dalloc<double>((size_t)h->grid_bnd_line, &st);
  h->counters = dalloc<unsigned>(8, &st);
  h->sc = dalloc<DevScalars>(1, &st);
  h->gam = dalloc<double>(kGamCap, &st);
  double *Hd = nullptr, *dd = nullptr;
  int *dcols = nullptr;
  Hd = dalloc<double>((size_t)nl * nb, &st);
  dd = dalloc<double>(nb, &st);
  dcols = dalloc<int>(nc, &st);
  auto cleanup_tmp = [&]() {
    if (Hd) (void)hipFree(Hd);
    if (dd) (void)hipFree(dd);
    if (dcols) (void)hipFree(dcols);
  };
  if (st != DCOPF_OK) {
    cleanup_tmp();
    free_handle(h);
    set_error("device allocation failed");
    return st;
  }
  hipStream_t s = h->stream;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (r != hipSuccess && e == hipSuccess) e = r;
  };
  chk(hipMemcpyAsync(Hd, p->H, (size_t)nl * nb * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(dd, p->d, (size_t)nb * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(dcols, cols.data(), (size_t)nc * 4, hipMemcpyHostToDevice, s));
  std::vector<double> qh(ng, 0.0);
  if (p->q) std::copy(p->q, p->q + ng, qh.begin());
  chk(hipMemcpyAsync(h->c, p->c, ng * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->q, qh.data(), ng * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->pmin, p->p_min, ng * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->pmax, p->p_max, ng * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->fmax, p->f_max, nl * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->seg, seg.data(), (nc + 1) * 4, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->gperm, gperm.data(), ng * 4, hipMemcpyHostToDevice, s));
  for (double **sp : state) chk(hipMemsetAsync(*sp, 0, nl * 8, s));
  chk(hipMemsetAsync(h->xbuf, 0, (size_t)h->ldc * esz, s));
  chk(hipMemsetAsync(h->counters, 0, 8 * sizeof(unsigned), s));
  chk(hipMemsetAsync(h->gam, 0, kGamCap * 8, s));
  DevScalars sch{};
  double D = 0.0;
  for (int b = 0; b < nb; ++b) D += p->d[b];
  sch.D = D;
  chk(hipMemcpyAsync(h->sc, &sch, sizeof(sch), hipMemcpyHostToDevice, s));
  // panels
  {
    dim3 gg((unsigned)std::min<int64_t>(64, (h->ldc + 255) / 256), (unsigned)nl);
    // the transposed panels are written over their full padded width ldl
    dim3 tg((unsigned)(h->ldc / 32), (unsigned)(h->ldl / 32));
    if (fp32) {
      gather_kernel<float><<<gg, 256, 0, s>>>(Hd, nb, nl, dcols, nc, h->ldc, h->P32);
      transpose_kernel<float><<<tg, dim3(32, 8), 0, s>>>(h->P32, nl, h->ldc, nc, h->ldl, h->P32T);
      // FP64 panel for the bound, transposed: gather into the (free) T slot first
      double *tmp = nullptr;
      chk(hipMalloc(&tmp, panel * 8));
      if (tmp) {
        gather_kernel<double><<<gg, 256, 0, s>>>(Hd, nb, nl, dcols, nc, h->ldc, tmp);
        transpose_kernel<double><<<tg, dim3(32, 8), 0, s>>>(tmp, nl, h->ldc, nc, h->ldl, h->P64T);
        chk(hipStreamSynchronize(s));
        (void)hipFree(tmp);
      }
    } else {
      gather_kernel<double><<<gg, 256, 0, s>>>(Hd, nb, nl, dcols, nc, h->ldc, h->P64);
      transpose_kernel<double><<<tg, dim3(32, 8), 0, s>>>(h->P64, nl, h->ldc, nc, h->ldl, h->P64T);
    }
    hd_kernel<<<grid_for(nl, 4, 4096), 256, 0, s>>>(Hd, nb, nl, dd, h->fd);
  }
  chk(hipGetLastError());
  refresh_v(h);
  chk(hipGetLastError());
  chk(hipStreamSynchronize(s));
  cleanup_tmp();
  if (e != hipSuccess) {
    set_error(std::string("HIP error during setup: ") + hipGetErrorString(e));
    free_handle(h);
    return DCOPF_E_HIP;
  }
  // largest possible cost (for the infeasibility certificate)
  double ub = 0.0;
  for (int g = 0; g < ng; ++g) {
    const double qq = p->q ? p->q[g] : 0.0;
    const double a = p->c[g] * p->p_min[g] + qq * p->p_min[g] * p->p_min[g];
    const double b = p->c[g] * p->p_max[g] + qq * p->p_max[g] * p->p_max[g];
    ub += std::max(a, b);
  }
  h->cost_ub = ub;
  // capture graph_iters iterations into a HIP graph (on a private stream)
  if (o->graph_iters > 0) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      free_handle(h);
      return set_error("hipStreamCreate failed"), DCOPF_E_HIP;
    }
    hipError_t ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (ce == hipSuccess) {
      launch_iters(h, cs, o->graph_iters);
      ce = hipStreamEndCapture(cs, &h->graph);
    }
    if (ce == hipSuccess) ce = hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (ce != hipSuccess) {
      set_error(std::string("graph capture failed: ") + hipGetErrorString(ce));
      free_handle(h);
      return DCOPF_E_HIP;
    }
  }
  *out = h;
  return DCOPF_OK;
}

dcopf_status dcopf_dual_step(dcopf_dual_t h, int64_t n) {
  if (!h || n < 0) return set_error("null handle or n < 0"), DCOPF_E_INVALID;
  int64_t left = n;
  if (h->graph_exec) {
    const int gi = h->opts.graph_iters;
    while (left >= gi) {
      DCOPF_HIP_TRY(hipGraphLaunch(h->graph_exec, h->stream));
      left -= gi;
    }
  }
  launch_iters(h, h->stream, left);
  DCOPF_HIP_TRY(hipGetLastError());
  h->iters += n;
  return DCOPF_OK;
}

static dcopf_status eval_bound(dcopf_dual_t h, double *value) {
  hipStream_t s = h->stream;
  const int blocks = (int)std::min<int64_t>(1024, (h->ldl + 255) / 256);
  make_v_kernel<double><<<blocks, 256, 0, s>>>(h->mu_p, h->mu_m, h->n_lines, h->ldl, h->v64b);
  StepParams none = h->prm;
  if (h->stage_bnd)
    colpass_kernel<double, false, true><<<h->grid_bnd_col, 256, h->lds_bnd, s>>>(
        h->P64T, h->n_cols, h->ldl, h->v64b, h->seg, h->gperm, h->c, h->q, h->pmin, h->pmax,
        h->sc, nullptr, h->part_a, h->counters + 2, none);
  else
    colpass_kernel<double, false, false><<<h->grid_bnd_col, 256, 0, s>>>(
        h->P64T, h->n_cols, h->ldl, h->v64b, h->seg, h->gperm, h->c, h->q, h->pmin, h->pmax,
        h->sc, nullptr, h->part_a, h->counters + 2, none);
  bound_lines_kernel<<<h->grid_bnd_line, 256, 0, s>>>(h->mu_p, h->mu_m, h->fd, h->fmax,
                                                       h->n_lines, h->sc, h->part_c,
                                                       h->counters + 3);
  DCOPF_HIP_TRY(hipGetLastError());
  DevScalars sch;
  DCOPF_HIP_TRY(hipMemcpyAsync(&sch, h->sc, sizeof(sch), hipMemcpyDeviceToHost, s));
  DCOPF_HIP_TRY(hipStreamSynchronize(s));
  *value = sch.bound_value;
  if (!std::isfinite(sch.bound_value) || !std::isfinite(sch.lam))
    return set_error("non-finite dual value or multiplier"), DCOPF_E_NONFINITE;
  if (sch.bound_value > h->best) {
    h->best = sch.bound_value;
    h->best_iter = h->iters;
  }
  return DCOPF_OK;
}

dcopf_status dcopf_dual_bound(dcopf_dual_t h, double *value, double *lambda, double *mu_plus,
                              double *mu_minus) {
  if (!h) return set_error("null handle"), DCOPF_E_INVALID;
  double v = NAN;
  dcopf_status st = eval_bound(h, &v);
  if (value) *value = v;
  if (lambda) {
    DevScalars sch;
    DCOPF_HIP_TRY(hipMemcpy(&sch, h->sc, sizeof(sch), hipMemcpyDeviceToHost));
    *lambda = sch.lam;
  }
  if (mu_plus) DCOPF_HIP_TRY(hipMemcpy(mu_plus, h->mu_p, h->n_lines * 8, hipMemcpyDeviceToHost));
  if (mu_minus)
    DCOPF_HIP_TRY(hipMemcpy(mu_minus, h->mu_m, h->n_lines * 8, hipMemcpyDeviceToHost));
  return st;
}

dcopf_status dcopf_dual_best(dcopf_dual_t h, double *value, int64_t *iteration) {
  if (!h) return set_error("null handle"), DCOPF_E_INVALID;
  if (value) *value = h->best;
  if (iteration) *iteration = h->best_iter;
  return DCOPF_OK;
}

dcopf_status dcopf_dual_gammas(dcopf_dual_t h, int64_t first, int64_t count, double *out) {
  if (!h || !out || first < 0 || count < 0)
    return set_error("bad arguments"), DCOPF_E_INVALID;
  if (first + count > h->iters || first < h->iters - kGamCap)
    return set_error("requested iterations not recorded"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(h->stream));
  for (int64_t i = 0; i < count;) {
    const int64_t k = (first + i) & (kGamCap - 1);
    const int64_t run = std::min<int64_t>(count - i, kGamCap - k);
    DCOPF_HIP_TRY(hipMemcpy(out + i, h->gam + k, run * 8, hipMemcpyDeviceToHost));
    i += run;
  }
  return DCOPF_OK;
}

dcopf_status dcopf_dual_solve(dcopf_dual_t h, double opt, double gap_tol, double dgamma_tol,
                              int64_t max_iters, int64_t check_every, dcopf_result *res) {
  if (!h || !res || max_iters < 0 || check_every < 1)
    return set_error("bad arguments"), DCOPF_E_INVALID;
  int64_t done = 0;
  int32_t status = 3;
  double val = NAN;
  const bool use_opt = std::isfinite(opt);
  dcopf_status st = eval_bound(h, &val);
  if (st != DCOPF_OK) return st;
  while (true) {
    if (use_opt && (opt - h->best) <= gap_tol * std::fabs(opt)) {
      status = 1;
      break;
    }
    if (h->best > h->cost_ub + 1e-9 * std::fabs(h->cost_ub))
      return set_error("dual bound exceeds the largest possible cost: infeasible"),
             DCOPF_E_INFEASIBLE;
    if (done >= max_iters) {
      status = 3;
      break;
    }
    const int64_t n = std::min<int64_t>(check_every, max_iters - done);
    st = dcopf_dual_step(h, n);
    if (st != DCOPF_OK) return st;
    done += n;
    st = eval_bound(h, &val);
    if (st != DCOPF_OK) return st;
    if (dgamma_tol > 0 && h->iters >= 2) {
      double g2[2];
      st = dcopf_dual_gammas(h, h->iters - 2, 2, g2);
      if (st != DCOPF_OK) return st;
      if (std::fabs(g2[1] - g2[0]) < dgamma_tol) {
        status = 2;
        break;
      }
    }
  }
  DevScalars sch;
  DCOPF_HIP_TRY(hipMemcpy(&sch, h->sc, sizeof(sch), hipMemcpyDeviceToHost));
  res->bound = h->best;
  res->gamma_last = sch.gamma_last;
  res->gap = use_opt ? (opt - h->best) / std::fabs(opt) : NAN;
  res->iters = h->iters;
  res->iter_of_bound = h->best_iter;
  res->status = status;
  return DCOPF_OK;
}

size_t dcopf_dual_state_len(dcopf_dual_t h) { return h ? 5 + 6 * (size_t)h->n_lines : 0; }

dcopf_status dcopf_dual_get_state(dcopf_dual_t h, double *buf, size_t len) {
  if (!h || !buf) return set_error("null argument"), DCOPF_E_INVALID;
  if (len != dcopf_dual_state_len(h)) return set_error("state length mismatch"), DCOPF_E_STATE;
  DCOPF_HIP_TRY(hipStreamSynchronize(h->stream));
  DevScalars sch;
  DCOPF_HIP_TRY(hipMemcpy(&sch, h->sc, sizeof(sch), hipMemcpyDeviceToHost));
  buf[0] = (double)sch.k;
  buf[1] = sch.lam;
  buf[2] = sch.v_lam;
  buf[3] = sch.s_lam;
  buf[4] = 0.0;
  const size_t nl = h->n_lines;
  double *arrs[] = {h->mu_p, h->mu_m, h->v_p, h->v_m, h->s_p, h->s_m};
  for (int i = 0; i < 6; ++i)
    DCOPF_HIP_TRY(hipMemcpy(buf + 5 + i * nl, arrs[i], nl * 8, hipMemcpyDeviceToHost));
  return DCOPF_OK;
}

dcopf_status dcopf_dual_set_state(dcopf_dual_t h, const double *buf, size_t len) {
  if (!h || !buf) return set_error("null argument"), DCOPF_E_INVALID;
  if (len != dcopf_dual_state_len(h)) return set_error("state length mismatch"), DCOPF_E_STATE;
  if (!finite_all(buf, len)) return set_error("non-finite state"), DCOPF_E_INVALID;
  const size_t nl = h->n_lines;
  for (size_t i = 0; i < 2 * nl; ++i)
    if (buf[5 + i] < 0.0) return set_error("mu must be >= 0"), DCOPF_E_INVALID;
  if (buf[0] < 0 || buf[0] != std::floor(buf[0]))
    return set_error("iteration must be a nonnegative integer"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(h->stream));
  DevScalars sch;
  DCOPF_HIP_TRY(hipMemcpy(&sch, h->sc, sizeof(sch), hipMemcpyDeviceToHost));
  sch.k = (long long)buf[0];
  sch.lam = buf[1];
  sch.v_lam = buf[2];
  sch.s_lam = buf[3];
  DCOPF_HIP_TRY(hipMemcpy(h->sc, &sch, sizeof(sch), hipMemcpyHostToDevice));
  double *arrs[] = {h->mu_p, h->mu_m, h->v_p, h->v_m, h->s_p, h->s_m};
  for (int i = 0; i < 6; ++i)
    DCOPF_HIP_TRY(hipMemcpy(arrs[i], buf + 5 + i * nl, nl * 8, hipMemcpyHostToDevice));
  h->iters = sch.k;
  refresh_v(h);
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(h->stream));
  return DCOPF_OK;
}

dcopf_status dcopf_dual_time_phases(dcopf_dual_t h, int64_t n, double *ms_out) {
  if (!h || !ms_out || n < 1) return set_error("bad arguments"), DCOPF_E_INVALID;
  std::vector<hipEvent_t> ev(4 * (size_t)n, nullptr);
  for (auto &e : ev) DCOPF_HIP_TRY(hipEventCreate(&e));
  for (int64_t i = 0; i < n; ++i) {
    for (int phase = 0; phase < 2; ++phase) {
      DCOPF_HIP_TRY(hipEventRecord(ev[4 * i + 2 * phase], h->stream));
      launch_phase(h, h->stream, phase);
      DCOPF_HIP_TRY(hipEventRecord(ev[4 * i + 2 * phase + 1], h->stream));
    }
  }
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(h->stream));
  double acc[2] = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i)
    for (int phase = 0; phase < 2; ++phase) {
      float ms = 0.f;
      DCOPF_HIP_TRY(hipEventElapsedTime(&ms, ev[4 * i + 2 * phase], ev[4 * i + 2 * phase + 1]));
      acc[phase] += ms;
    }
  for (auto &e : ev) (void)hipEventDestroy(e);
  ms_out[0] = acc[0] / n;
  ms_out[1] = acc[1] / n;
  h->iters += n;
  return DCOPF_OK;
}

dcopf_status dcopf_dual_info(dcopf_dual_t h, int32_t *n_cols, int64_t *iters) {
  if (!h) return set_error("null handle"), DCOPF_E_INVALID;
  if (n_cols) *n_cols = h->n_cols;
  if (iters) *iters = h->iters;
  return DCOPF_OK;
}

void dcopf_dual_destroy(dcopf_dual_t h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  free_handle(h);
}

}  // extern "C"
