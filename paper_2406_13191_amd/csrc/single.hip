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

thread_local DevMem g_mem;  // the allocator installed on this thread
DevMem current_devmem(void *stream) {
  DevMem m = g_mem;
  m.stream = stream;
  return m;
}

// Scalars of one iteration.  Two slots, indexed by the parity of the
// iteration, so a kernel can read the previous iteration's slot while its
// workgroup 0 writes the current one.
struct IterSlot {
  double lam, v_lam, s_lam;  // balance multiplier (and optimiser state) used
                             // by this iteration
  double alpha, c1, c2;      // step size and Adam bias corrections
  long long k;               // iteration index (-1 before the first)
  int pending;               // partial sums of this iteration not yet folded
  int pad;
};

struct DevScalars {
  IterSlot slot[2];
  double D;                  // 1^T d
  double gamma_last;         // monitor value of the last folded iterate
  double bound_gen, bound_value;
  long long avg_count;       // iterations summed into the primal average
  int avg_on;                // column passes add p* to the primal sum
  int avg_pad;
};

// Result of the primal evaluation (device side of dcopf_primal).
struct DevPrimal {
  double cost, balance, max_overload, sum_overload;
  long long count;
  int n_overloaded, pad;
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

// Finish iteration `prev` from its summed partials: its dual value
// gamma = sum phi + lambda D - line terms, and the lambda step with the
// balance residual D - sum p* (Algorithm 1 / Adam / AdaGrad).  Returns the
// slot of the next iteration (not yet pending).
__device__ __forceinline__ IterSlot fold(const IterSlot &prev, double psum, double phisum,
                                         double lines, double D, const StepParams &prm,
                                         double *gamma) {
  *gamma = phisum + prev.lam * D - lines;
  const double g = D - psum;
  const double a = prev.alpha;
  IterSlot n = prev;
  if (prm.rule == DCOPF_RULE_GDM) {
    n.v_lam = prm.rho * prev.v_lam + a * g;
    n.lam = prev.lam + n.v_lam;
    if (prm.literal) n.lam += a * g;
  } else if (prm.rule == DCOPF_RULE_ADAM) {
    n.v_lam = prm.beta1 * prev.v_lam + (1.0 - prm.beta1) * g;
    n.s_lam = prm.beta2 * prev.s_lam + (1.0 - prm.beta2) * g * g;
    n.lam = prev.lam + a * (n.v_lam / prev.c1) / (sqrt(n.s_lam / prev.c2) + prm.eps);
  } else {
    n.s_lam = prev.s_lam + g * g;
    n.lam = prev.lam + a * g / (sqrt(n.s_lam) + prm.eps);
  }
  n.pending = 0;
  return n;
}

// Step size and bias corrections of iteration k.
__device__ __forceinline__ void set_step(IterSlot &s, long long k, const StepParams &prm) {
  const double kk = (double)k;
  s.k = k;
  s.alpha = prm.decay == 0.0 ? prm.alpha : prm.alpha / (1.0 + prm.decay * kk);
  // Adam's bias corrections; pow is costly, the other rules skip it
  s.c1 = s.c2 = 1.0;
  if (prm.rule == DCOPF_RULE_ADAM) {
    s.c1 = 1.0 - pow(prm.beta1, kk + 1.0);
    s.c2 = 1.0 - pow(prm.beta2, kk + 1.0);
  }
}

// Sum (in index order, deterministic) the partials the previous iteration
// left: column-pass (sum p*, sum phi) pairs and line-pass line terms.
__device__ __forceinline__ void sum_partials(const double *pa, int ga, const double *pb, int gb,
                                             double *red, double *ps, double *phis,
                                             double *lines) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int b = threadIdx.x; b < ga; b += blockDim.x) {
    s0 += pa[2 * b];
    s1 += pa[2 * b + 1];
  }
  for (int b = threadIdx.x; b < gb; b += blockDim.x) s2 += pb[b];
  *ps = block_sum(s0, red);
  *phis = block_sum(s1, red);
  *lines = block_sum(s2, red);
}

// A 16-byte panel chunk.  Panels whose two orientations fit in the 256 MB
// last-level cache (MALL) are read with plain loads, which keep them there
// between iterations (a 112 MB panel: 10 % less time per iteration than
// nontemporal loads); larger panels are read nontemporally (a 508 MB panel:
// 8 % less than plain loads).
constexpr size_t kMallBytes = 256ull << 20;
template <bool NT, typename V> __device__ __forceinline__ V panel_ld(const V *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// Per-lane share of a row dot product: lane `lane` covers the 16-byte
// chunks lane, lane + 64, ... of a row of `nv` chunks.
template <typename T, bool NT>
__device__ __forceinline__ T lane_dot(const T *__restrict__ row, const T *__restrict__ x, int nv,
                                      int lane) {
  using V = typename Vec16<T>::type;
  const V *r = reinterpret_cast<const V *>(row);
  const V *xv = reinterpret_cast<const V *>(x);
  T a0 = 0, a1 = 0;
  int i = lane;
  for (; i + kWave < nv; i += 2 * kWave) {
    V p0 = panel_ld<NT>(r + i);
    V p1 = panel_ld<NT>(r + i + kWave);
    a0 = fma_vec(p0, xv[i], a0);
    a1 = fma_vec(p1, xv[i + kWave], a1);
  }
  if (i < nv) a0 = fma_vec(panel_ld<NT>(r + i), xv[i], a0);
  return a0 + a1;
}

template <typename T>
__device__ __forceinline__ void stage_vec(T *dst, const T *src, int ld) {
  using V = typename Vec16<T>::type;
  constexpr int NV = Vec16<T>::n;
  for (int i = threadIdx.x; i < ld / NV; i += blockDim.x)
    reinterpret_cast<V *>(dst)[i] = reinterpret_cast<const V *>(src)[i];
}

// Generators of panel column j handled lane-parallel: r, p*, phi per unit,
// wave sums of p* (the column injection) and phi.  Every lane gets the sums.
// Unit data is stored column-sorted: the units of column j are
// seg[j] .. seg[j+1] - 1.
// Units of column j handled lane-parallel by one wavefront: lane l takes
// units g0 + l, g0 + l + 64, ...  The data of the lane's first unit (cf, qf,
// lof, hif; valid when g0 + lane < g1) were loaded earlier.
// With sd (the iterated-s dual): a unit's s and its velocity in sd[0][t],
// sd[1][t]; the unit is bang-bang on the shifted cost and s takes its GDM
// step (alpha, rho) here, its owner lane being the only one to touch it.
struct SDual {
  double *s, *v;
};

__device__ __forceinline__ void column_units(double w, double lam, int g0, int g1, double cf,
                                             double qf, double lof, double hif,
                                             const double *__restrict__ c,
                                             const double *__restrict__ q,
                                             const double *__restrict__ pmin,
                                             const double *__restrict__ pmax, int lane,
                                             double *xj, double *phij,
                                             double *__restrict__ psum = nullptr,
                                             SDual sd = SDual{nullptr, nullptr},
                                             double alpha = 0.0, double rho = 0.0) {
  double xs = 0.0, ph = 0.0;
  for (int t = g0 + lane; t < g1; t += kWave) {
    const bool first = t == g0 + lane;
    const double ct = first ? cf : c[t], qt = first ? qf : q[t];
    const double lo = first ? lof : pmin[t], hi = first ? hif : pmax[t];
    const double r = ct - lam + w;
    double p;
    if (sd.s) {
      // Section 3.2, eq. QP_finalgamma with s fixed: q (p - m)^2 is bounded
      // below by -sqrt(q) s (p - m) - s^2 / 4
      const double m = 0.5 * (lo + hi), sq = sqrt(qt), st = sd.s[t];
      const double a = r + 2.0 * qt * m - sq * st;
      p = inner_min(a, 0.0, lo, hi);
      ph += a * p - qt * m * m + sq * st * m - 0.25 * st * st;
      const double v = rho * sd.v[t] + alpha * (-sq * (p - m) - 0.5 * st);
      sd.v[t] = v;
      sd.s[t] = st + v;
    } else {
      p = inner_min(r, qt, lo, hi);
      ph += r * p + qt * p * p;
    }
    xs += p;
    if (psum) psum[t] += p;  // primal average (each unit has one owner lane)
  }
  *xj = wave_sum(xs);
  *phij = wave_sum(ph);
}

// The same for column j, loading everything here.
__device__ __forceinline__ void column_units(int j, double w, double lam,
                                             const int *__restrict__ seg,
                                             const double *__restrict__ c,
                                             const double *__restrict__ q,
                                             const double *__restrict__ pmin,
                                             const double *__restrict__ pmax, int lane,
                                             double *xj, double *phij) {
  const int g0 = seg[j], g1 = seg[j + 1];
  const int tf = g0 + lane < g1 ? g0 + lane : 0;
  column_units(w, lam, g0, g1, c[tf], q[tf], pmin[tf], pmax[tf], c, q, pmin, pmax, lane, xj,
               phij);
}

// Partials of a previous launch, n of them (index idx, element a[idx *
// stride + off]), summed over the workgroup's threads (idx = threadIdx.x +
// m blockDim.x).  load() issues the first kPre loads from clamped indices
// without waiting; sum() adds them and any further terms.
constexpr int kPre = 4;
struct StridedSum {
  double v[kPre];
  __device__ __forceinline__ void load(const double *__restrict__ a, int n, int stride, int off) {
#pragma unroll
    for (int m = 0; m < kPre; ++m) {
      const int idx = threadIdx.x + m * blockDim.x;
      v[m] = ldg(a + (size_t)(idx < n ? idx : 0) * stride + off);
    }
  }
  __device__ __forceinline__ double sum(const double *__restrict__ a, int n, int stride,
                                        int off) const {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < kPre; ++m)
      if ((int)(threadIdx.x + m * blockDim.x) < n) s += v[m];
    for (int idx = threadIdx.x + kPre * blockDim.x; idx < n; idx += blockDim.x)
      s += a[(size_t)idx * stride + off];
    return s;
  }
};

// ---------------------------------------------------------------------------
// Column pass of iteration k (parity par = k & 1).  A workgroup owns CB
// panel columns; its four wavefronts each stream one quarter of those rows
// of P^T (the matching quarter of v is read into registers once), and the
// quarter sums meet in LDS in a fixed order.  Every workgroup also folds
// iteration k-1 (identically, from its partials) to obtain the lambda of
// iteration k; workgroup 0 records it.  Wavefront c then handles the units
// of column c lane-parallel and writes the injection x_j.
//
// Memory round trips are the cost for panels of a few MB, so the loads are
// ordered by dependence: the unit boundaries first, then the partials of
// iteration k-1 and (UNR > 0: every chunk, at most UNR per lane) the panel
// and v chunks, then the data of each lane's first unit, which waits only
// for the boundaries.  UNR = 0 streams larger panels in a loop.
// ---------------------------------------------------------------------------
template <typename T, int CB, int UNR, bool NT>
__global__ __launch_bounds__(256) void colpass_kernel(
    const T *__restrict__ PT, int n_cols, int ldl, const T *__restrict__ vvec,
    const int *__restrict__ seg, const double *__restrict__ c, const double *__restrict__ q,
    const double *__restrict__ pmin, const double *__restrict__ pmax, DevScalars *sc, int par,
    T *__restrict__ x_out, double *__restrict__ part_a, int ga, const double *__restrict__ part_b,
    int gb, StepParams prm, double *__restrict__ gam_buf, long long gam_mask,
    double *__restrict__ psum, SDual sd) {
  using V = typename Vec16<T>::type;
  __shared__ double red[3 * 4];
  __shared__ double alpha_s;
  __shared__ double lam_s;
  __shared__ T dots[4][CB];
  __shared__ double colsum[2][4];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int j0 = blockIdx.x * CB;
  // (1) units of this wavefront's column (wavefronts c < CB own column j0 + c)
  const bool unit_wave = wave < CB && j0 + wave < n_cols;
  const int jw = unit_wave ? j0 + wave : 0;
  const int g0 = ldg(seg + jw), g1 = ldg(seg + jw + 1);
  // (2) the previous iteration's partials (loaded whether or not they are
  // pending: the buffers always exist; unused values are dropped)
  const IterSlot prev = sc->slot[par ^ 1];
  const double *pa = part_a + (size_t)(par ^ 1) * 2 * ga;
  const double *pb = part_b + (size_t)(par ^ 1) * gb;
  StridedSum f0, f1, f2;
  f0.load(pa, ga, 2, 0);
  f1.load(pa, ga, 2, 1);
  f2.load(pb, gb, 1, 0);
  // (3) quarter of every owned row: chunks [cb, ce) of nv 16-byte chunks
  const int nv = ldl / Vec16<T>::n;
  const int quarter = (nv + 3) / 4;
  const int cb = wave * quarter, ce = min(nv, cb + quarter);
  const V *vv = reinterpret_cast<const V *>(vvec);
  T acc[CB];
#pragma unroll
  for (int u = 0; u < CB; ++u) acc[u] = (T)0;
  const V *rows[CB];
#pragma unroll
  for (int u = 0; u < CB; ++u)
    rows[u] = reinterpret_cast<const V *>(PT + (size_t)min(j0 + u, n_cols - 1) * ldl);
  double cf = 0.0, qf = 0.0, lof = 0.0, hif = 0.0;
  const int tf = g0 + lane < g1 ? g0 + lane : 0;
  if (UNR > 0) {
    V pv[UNR > 0 ? UNR : 1][CB], xv[UNR > 0 ? UNR : 1];
#pragma unroll
    for (int m = 0; m < UNR; ++m) {
      const int i = cb + lane + m * kWave;
      const int ic = i < ce ? i : 0;
      xv[m] = vv[ic];
#pragma unroll
      for (int u = 0; u < CB; ++u) pv[m][u] = panel_ld<NT>(rows[u] + ic);
    }
    // (4) the lane's first unit: waits for the boundaries only
    cf = ldg(c + tf);
    qf = ldg(q + tf);
    lof = ldg(pmin + tf);
    hif = ldg(pmax + tf);
#pragma unroll
    for (int m = 0; m < UNR; ++m)
      if (cb + lane + m * kWave < ce)
#pragma unroll
        for (int u = 0; u < CB; ++u) acc[u] = fma_vec(pv[m][u], xv[m], acc[u]);
  } else {
    // streamed: four chunks of every owned row per lane and iteration, all
    // loaded before they are used
    T acc2[CB], acc3[CB], acc4[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) acc2[u] = acc3[u] = acc4[u] = (T)0;
    int i = cb + lane;
    for (; i + 3 * kWave < ce; i += 4 * kWave) {
      V x[4], p[4][CB];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        x[m] = vv[i + m * kWave];
#pragma unroll
        for (int u = 0; u < CB; ++u) p[m][u] = panel_ld<NT>(rows[u] + i + m * kWave);
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        acc[u] = fma_vec(p[0][u], x[0], acc[u]);
        acc2[u] = fma_vec(p[1][u], x[1], acc2[u]);
        acc3[u] = fma_vec(p[2][u], x[2], acc3[u]);
        acc4[u] = fma_vec(p[3][u], x[3], acc4[u]);
      }
    }
    for (; i < ce; i += kWave) {
      const V x0 = vv[i];
#pragma unroll
      for (int u = 0; u < CB; ++u)
        acc[u] = fma_vec(panel_ld<NT>(rows[u] + i), x0, acc[u]);
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) acc[u] = (acc[u] + acc2[u]) + (acc3[u] + acc4[u]);
    cf = ldg(c + tf);
    qf = ldg(q + tf);
    lof = ldg(pmin + tf);
    hif = ldg(pmax + tf);
  }
#pragma unroll
  for (int u = 0; u < CB; ++u) {
    const T d = wave_sum(acc[u]);
    if (lane == 0) dots[wave][u] = d;
  }
  double fsum[3] = {0.0, 0.0, 0.0};
  if (prev.pending) {
    fsum[0] = f0.sum(pa, ga, 2, 0);
    fsum[1] = f1.sum(pa, ga, 2, 1);
    fsum[2] = f2.sum(pb, gb, 1, 0);
    block_sums<3>(fsum, red);
  }
  const double ps = fsum[0], phis = fsum[1], lines = fsum[2];
  if (threadIdx.x == 0) {
    IterSlot cur = prev;
    double gam = 0.0;
    if (prev.pending) cur = fold(prev, ps, phis, lines, sc->D, prm, &gam);
    set_step(cur, prev.k + 1, prm);
    cur.pending = 1;
    lam_s = cur.lam;
    alpha_s = cur.alpha;
    if (blockIdx.x == 0) {
      sc->slot[par] = cur;
      if (prev.pending) {
        gam_buf[prev.k & gam_mask] = gam;
        sc->gamma_last = gam;
      }
      if (sc->avg_on) sc->avg_count += 1;
    }
  }
  __syncthreads();
  double xsum = 0.0, phsum = 0.0;
  if (unit_wave) {
    const double w = (double)(((dots[0][wave] + dots[1][wave]) + dots[2][wave]) + dots[3][wave]);
    double xj, phij;
    column_units(w, lam_s, g0, g1, cf, qf, lof, hif, c, q, pmin, pmax, lane, &xj, &phij,
                 sc->avg_on ? psum : nullptr, sd, alpha_s, prm.rho);
    if (lane == 0) x_out[jw] = (T)xj;
    xsum = xj;
    phsum = phij;
  }
  if (lane == 0) {
    colsum[0][wave] = xsum;
    colsum[1][wave] = phsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part_a[(size_t)par * 2 * ga + 2 * blockIdx.x] =
        ((colsum[0][0] + colsum[0][1]) + colsum[0][2]) + colsum[0][3];
    part_a[(size_t)par * 2 * ga + 2 * blockIdx.x + 1] =
        ((colsum[1][0] + colsum[1][1]) + colsum[1][2]) + colsum[1][3];
  }
}

// Sums of the previous iteration's partials taken by one wavefront: lane l
// adds the entries l, l + 64, ... (the first kPreW of them loaded before any
// wait by load()), then the lanes' sums meet in a butterfly.  The finalize
// kernel uses the same order when the column pass does (bitwise equal
// results however the iterations are split into calls).
constexpr int kPreW = 16;
struct WaveSums {
  double a0[kPreW], a1[kPreW], b0[kPreW];
  __device__ __forceinline__ void load(const double *__restrict__ pa, int ga,
                                       const double *__restrict__ pb, int gb, int lane) {
#pragma unroll
    for (int m = 0; m < kPreW; ++m) {
      const int ia = lane + m * kWave, ib = lane + m * kWave;
      a0[m] = ldg(pa + 2 * (size_t)(ia < ga ? ia : 0));
      a1[m] = ldg(pa + 2 * (size_t)(ia < ga ? ia : 0) + 1);
      b0[m] = ldg(pb + (ib < gb ? ib : 0));
    }
  }
  __device__ __forceinline__ void sum(const double *__restrict__ pa, int ga,
                                      const double *__restrict__ pb, int gb, int lane,
                                      double *ps, double *phis, double *lines) const {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int m = 0; m < kPreW; ++m) {
      if (lane + m * kWave < ga) {
        s0 += a0[m];
        s1 += a1[m];
      }
      if (lane + m * kWave < gb) s2 += b0[m];
    }
    for (int i = lane + kPreW * kWave; i < ga; i += kWave) {
      s0 += pa[2 * (size_t)i];
      s1 += pa[2 * (size_t)i + 1];
    }
    for (int i = lane + kPreW * kWave; i < gb; i += kWave) s2 += pb[i];
    *ps = wave_sum(s0);
    *phis = wave_sum(s1);
    *lines = wave_sum(s2);
  }
};

// ---------------------------------------------------------------------------
// Column pass with one column per workgroup (panels of at most 8 chunks per
// lane and quarter): one barrier in all.  The four wavefronts each load and
// multiply a quarter of the column against v; wavefront 0 meanwhile loads the
// column's units and every partial of iteration k-1.  After the quarter sums
// meet in LDS, wavefront 0 alone folds iteration k-1 (lane-parallel, no
// further barrier), runs the units and writes x_j and the workgroup's
// partials; workgroup 0 records the new slot.
// ---------------------------------------------------------------------------
template <typename T, int UNR>
__global__ __launch_bounds__(256) void colpass1_kernel(
    const T *__restrict__ PT, int n_cols, int ldl, const T *__restrict__ vvec,
    const int *__restrict__ seg, const double *__restrict__ c, const double *__restrict__ q,
    const double *__restrict__ pmin, const double *__restrict__ pmax, DevScalars *sc, int par,
    T *__restrict__ x_out, double *__restrict__ part_a, int ga, const double *__restrict__ part_b,
    int gb, StepParams prm, double *__restrict__ gam_buf, long long gam_mask,
    double *__restrict__ psum, SDual sd) {
  using V = typename Vec16<T>::type;
  __shared__ T dots[4];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int j = blockIdx.x;
  const IterSlot prev = sc->slot[par ^ 1];
  const double *pa = part_a + (size_t)(par ^ 1) * 2 * ga;
  const double *pb = part_b + (size_t)(par ^ 1) * gb;
  // wavefront 0: the column's unit boundaries and the previous partials
  int g0 = 0, g1 = 0;
  WaveSums ws;
  if (wave == 0) {
    g0 = ldg(seg + j);
    g1 = ldg(seg + j + 1);
    ws.load(pa, ga, pb, gb, lane);
  }
  // every wavefront: a quarter of the column (all chunks in flight at once)
  const int nv = ldl / Vec16<T>::n;
  const int quarter = (nv + 3) / 4;
  const int cb = wave * quarter, ce = min(nv, cb + quarter);
  const V *vv = reinterpret_cast<const V *>(vvec);
  const V *row = reinterpret_cast<const V *>(PT + (size_t)j * ldl);
  V pv[UNR], xv[UNR];
#pragma unroll
  for (int m = 0; m < UNR; ++m) {
    const int i = cb + lane + m * kWave;
    const int ic = i < ce ? i : 0;
    xv[m] = vv[ic];
    pv[m] = panel_ld<false>(row + ic);
  }
  // wavefront 0: the lane's first unit (waits for the boundaries only)
  double cf = 0.0, qf = 0.0, lof = 0.0, hif = 0.0;
  if (wave == 0) {
    const int tf = g0 + lane < g1 ? g0 + lane : 0;
    cf = ldg(c + tf);
    qf = ldg(q + tf);
    lof = ldg(pmin + tf);
    hif = ldg(pmax + tf);
  }
  T acc = (T)0;
#pragma unroll
  for (int m = 0; m < UNR; ++m)
    if (cb + lane + m * kWave < ce) acc = fma_vec(pv[m], xv[m], acc);
  const T d = wave_sum(acc);
  if (lane == 0) dots[wave] = d;
  __syncthreads();
  if (wave != 0) return;
  // wavefront 0: fold iteration k-1, then the units of column j
  IterSlot cur = prev;
  if (prev.pending) {
    double ps, phis, lines, gam;
    ws.sum(pa, ga, pb, gb, lane, &ps, &phis, &lines);
    cur = fold(prev, ps, phis, lines, sc->D, prm, &gam);
    if (blockIdx.x == 0 && lane == 0) {
      gam_buf[prev.k & gam_mask] = gam;
      sc->gamma_last = gam;
    }
  }
  set_step(cur, prev.k + 1, prm);
  cur.pending = 1;
  const bool avg = sc->avg_on;
  if (blockIdx.x == 0 && lane == 0) {
    sc->slot[par] = cur;
    if (avg) sc->avg_count += 1;
  }
  const double w = (double)(((dots[0] + dots[1]) + dots[2]) + dots[3]);
  double xj, phij;
  column_units(w, cur.lam, g0, g1, cf, qf, lof, hif, c, q, pmin, pmax, lane, &xj, &phij,
               avg ? psum : nullptr, sd, cur.alpha, prm.rho);
  if (lane == 0) {
    x_out[j] = (T)xj;
    part_a[(size_t)par * 2 * ga + 2 * j] = xj;
    part_a[(size_t)par * 2 * ga + 2 * j + 1] = phij;
  }
}

// ---------------------------------------------------------------------------
// Line pass of iteration k: F = P x - f_d for RW lines per wavefront (their
// loads interleaved), then lane t < RW applies the step and projection to
// line t (its state was prefetched before the products), writes the next v,
// and the line terms of gamma_k go to a per-workgroup partial.
// ---------------------------------------------------------------------------
template <typename T, bool STAGE, int RW, int XR, bool NT>
__global__ __launch_bounds__(256) void linepass_kernel(
    const T *__restrict__ P, int n_lines, int ldc, const T *__restrict__ x_in,
    const double *__restrict__ fd, const double *__restrict__ flim,
    double *__restrict__ mu_p, double *__restrict__ mu_m, double *__restrict__ v_p,
    double *__restrict__ v_m, double *__restrict__ s_p, double *__restrict__ s_m,
    T *__restrict__ v_out, const DevScalars *sc, int par, double *__restrict__ part_b, int gb,
    StepParams prm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int base = (blockIdx.x * nw + wave) * RW;
  // prefetch the state of line base + lane
  const int l = base + lane;
  const bool mine = lane < RW && l < n_lines;
  const int lc = mine ? l : 0;  // loads from a valid line; results kept only when mine
  double fdl = ldg(fd + lc), fl = ldg(flim + lc), mp = ldg(mu_p + lc), mm = ldg(mu_m + lc),
         vp = ldg(v_p + lc), vm = ldg(v_m + lc), sp = 0, sm = 0;
  if (prm.rule != DCOPF_RULE_GDM) {
    sp = ldg(s_p + lc);
    sm = ldg(s_m + lc);
  }
  const IterSlot cur = sc->slot[par];
  const int nv = ldc / Vec16<T>::n;
  T acc[RW];
  if (XR > 0) {
    // narrow panel: the x chunks this lane needs (the same for every row)
    // are held in registers, no LDS staging and no barrier
    // Every load is issued from a clamped (in-range) index before the first
    // wait; out-of-range terms are masked afterwards.
    using V = typename Vec16<T>::type;
    const V *xv = reinterpret_cast<const V *>(x_in);
    V xr[XR > 0 ? XR : 1], pr[RW][XR > 0 ? XR : 1];
#pragma unroll
    for (int u = 0; u < XR; ++u) {
      const int idx = lane + u * kWave;
      xr[u] = xv[idx < nv ? idx : 0];
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const V *row = reinterpret_cast<const V *>(P + (size_t)min(base + r, n_lines - 1) * ldc);
#pragma unroll
      for (int u = 0; u < XR; ++u) {
        const int idx = lane + u * kWave;
        pr[r][u] = panel_ld<NT>(row + (idx < nv ? idx : 0));
      }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      T a = (T)0;
#pragma unroll
      for (int u = 0; u < XR; ++u)
        if (lane + u * kWave < nv) a = fma_vec(pr[r][u], xr[u], a);
      acc[r] = base + r < n_lines ? a : (T)0;
    }
  } else {
    const T *xs = x_in;
    if (STAGE) {
      stage_vec(reinterpret_cast<T *>(smem_raw), x_in, ldc);
      __syncthreads();
      xs = reinterpret_cast<const T *>(smem_raw);
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
      acc[r] = (base + r < n_lines) ? lane_dot<T, NT>(P + (size_t)(base + r) * ldc, xs, nv, lane)
                                    : (T)0;
  }
  double dot = 0.0;
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const T s = wave_sum(acc[r]);
    if (lane == r) dot = (double)s;
  }
  double term = 0.0;
  if (mine) {
    const double F = dot - fdl;
    const double gp = F - fl, gm = -F - fl;
    term = (mp - mm) * fdl + (mp + mm) * fl;
    const double a = cur.alpha;
    double np_, nm_;
    if (prm.rule == DCOPF_RULE_GDM) {
      vp = prm.rho * vp + a * gp;
      vm = prm.rho * vm + a * gm;
      v_p[l] = vp;
      v_m[l] = vm;
      np_ = mp + vp;
      nm_ = mm + vm;
      if (prm.literal) {
        np_ += a * gp;
        nm_ += a * gm;
      }
    } else if (prm.rule == DCOPF_RULE_ADAM) {
      vp = prm.beta1 * vp + (1.0 - prm.beta1) * gp;
      vm = prm.beta1 * vm + (1.0 - prm.beta1) * gm;
      sp = prm.beta2 * sp + (1.0 - prm.beta2) * gp * gp;
      sm = prm.beta2 * sm + (1.0 - prm.beta2) * gm * gm;
      v_p[l] = vp;
      v_m[l] = vm;
      s_p[l] = sp;
      s_m[l] = sm;
      np_ = mp + a * (vp / cur.c1) / (sqrt(sp / cur.c2) + prm.eps);
      nm_ = mm + a * (vm / cur.c1) / (sqrt(sm / cur.c2) + prm.eps);
    } else {
      sp += gp * gp;
      sm += gm * gm;
      s_p[l] = sp;
      s_m[l] = sm;
      np_ = mp + a * gp / (sqrt(sp) + prm.eps);
      nm_ = mm + a * gm / (sqrt(sm) + prm.eps);
    }
    np_ = fmax(np_, 0.0);
    nm_ = fmax(nm_, 0.0);
    mu_p[l] = np_;
    mu_m[l] = nm_;
    v_out[l] = (T)(np_ - nm_);
  }
  // one partial per wavefront (no workgroup barrier)
  const double wl = wave_sum(term);
  if (lane == 0) part_b[(size_t)par * gb + blockIdx.x * nw + wave] = wl;
}

// Fold the last iteration of a step() call (one workgroup).
__global__ __launch_bounds__(256) void finalize_kernel(DevScalars *sc, int par,
                                                       const double *__restrict__ part_a, int ga,
                                                       const double *__restrict__ part_b, int gb,
                                                       StepParams prm,
                                                       double *__restrict__ gam_buf,
                                                       long long gam_mask, int wave_order) {
  __shared__ double red[4];
  const IterSlot s = sc->slot[par];
  if (!s.pending) return;
  double ps, phis, lines;
  if (wave_order) {
    // the summation order of the one-column column pass
    if (threadIdx.x >= kWave) return;
    WaveSums ws;
    const double *pa = part_a + (size_t)par * 2 * ga, *pb = part_b + (size_t)par * gb;
    ws.load(pa, ga, pb, gb, threadIdx.x);
    ws.sum(pa, ga, pb, gb, threadIdx.x, &ps, &phis, &lines);
  } else {
    sum_partials(part_a + (size_t)par * 2 * ga, ga, part_b + (size_t)par * gb, gb, red, &ps,
                 &phis, &lines);
  }
  if (threadIdx.x == 0) {
    double gam = 0.0;
    IterSlot n = fold(s, ps, phis, lines, sc->D, prm, &gam);
    sc->slot[par] = n;  // same iteration index, lambda advanced, not pending
    gam_buf[s.k & gam_mask] = gam;
    sc->gamma_last = gam;
  }
}

// ---------------------------------------------------------------------------
// Read-once iteration (panels whose rows fit the registers of a workgroup).
// The two products of an iteration share one read of P (row-major):
//
//   line pass of iteration k:  per line l, F_l = P_l x - f_d,l, the residuals
//       and the step and projection of mu_l, then with the same row of P
//       still in registers the line's contribution P_l^T v_l of the new
//       v_l = mu+_l - mu-_l to the next iteration's reduced costs;
//       workgroup g writes its sum over its lines as the partial W_g of
//       w = P^T v (columns in its lanes, fixed order);
//   unit pass of iteration k+1: w = sum_g W_g (index order, FP64), then the
//       units (reduced cost, inner minimiser, x) as in the column pass.
//
// So each iteration reads the panel once instead of once per orientation;
// the partials (workgroups x columns) are the price.  A workgroup owns a
// contiguous range of lines; its waves form 4 / QW row groups of QW waves,
// each wave covering a slice of every row's 16-byte chunks (CPL per lane),
// and a row group takes RW rows at a time.  With QW > 1 the slices' dot
// products meet in LDS (one barrier per RW rows).  x stays in registers;
// the w partials are accumulated in registers and the row groups' sums meet
// in LDS at the end.
//
// With prime = 1 the pass only forms the partials of the current v (after
// the state was set); the arithmetic is that of a step, so a resumed run is
// bitwise equal to an uninterrupted one.
// ---------------------------------------------------------------------------
template <typename V, typename T> __device__ __forceinline__ V axpy_vec(const V &p, T v, V acc);
template <> __device__ __forceinline__ f32x4 axpy_vec(const f32x4 &p, float v, f32x4 acc) {
  acc.x = fmaf(p.x, v, acc.x);
  acc.y = fmaf(p.y, v, acc.y);
  acc.z = fmaf(p.z, v, acc.z);
  acc.w = fmaf(p.w, v, acc.w);
  return acc;
}
template <> __device__ __forceinline__ f64x2 axpy_vec(const f64x2 &p, double v, f64x2 acc) {
  acc.x = fma(p.x, v, acc.x);
  acc.y = fma(p.y, v, acc.y);
  return acc;
}

// Rows of one block: the panel chunks and the state of line (first row +
// lane) for lanes < RW.
template <typename V, int RW, int CPL> struct RowBlock {
  V pr[RW][CPL];
  double mp, mm, fdl, fl, vp, vm, sp, sm;
};

template <typename T, int QW, int RW, int CPL, bool NT, bool PIPE>
__global__ __launch_bounds__(256) void rlines_kernel(
    const T *__restrict__ P, int n_lines, int ldc, const T *__restrict__ x_in,
    const double *__restrict__ fd, const double *__restrict__ flim,
    double *__restrict__ mu_p, double *__restrict__ mu_m, double *__restrict__ v_p,
    double *__restrict__ v_m, double *__restrict__ s_p, double *__restrict__ s_m,
    const DevScalars *sc, int par, double *__restrict__ part_b, int gb,
    T *__restrict__ part_w, StepParams prm, int prime) {
  using V = typename Vec16<T>::type;
  using Blk = RowBlock<V, RW, CPL>;
  constexpr int VN = Vec16<T>::n;
  constexpr int NRG = 4 / QW;
  extern __shared__ __align__(16) unsigned char smem_raw[];  // [NRG - 1][ldc] of T
  __shared__ T dots[2][NRG][RW][QW];
  // the wavefront index is uniform: in a scalar register, so row addresses
  // are scalar bases with per-lane offsets
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int rg = wave / QW, qi = wave % QW;
  const int nv = ldc / VN;
  const int qc = (nv + QW - 1) / QW;
  const int c0 = qi * qc, c1 = min(nv, c0 + qc);
  // contiguous, balanced line ranges (every workgroup has at least one line)
  const int l_begin = (int)((long long)blockIdx.x * n_lines / gridDim.x);
  const int l_end = (int)((long long)(blockIdx.x + 1) * n_lines / gridDim.x);
  const int nblk = (l_end - l_begin + RW - 1) / RW;
  // chunk indices of this lane (clamped to a valid chunk; masked by xr = 0
  // in the dot products and never stored)
  unsigned cidx[CPL];  // unsigned: a scalar row base plus a 32-bit lane offset
  bool cval[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    const int i = c0 + lane + u * kWave;
    cval[u] = i < c1;
    cidx[u] = cval[u] ? (unsigned)i : 0u;
  }
  // Block bb of this row group: its rows (rows past the range read a valid
  // row and get weight 0) and the state of its line lane < RW.
  auto load_blk = [&](int bb, Blk &B) {
    const int b = bb + rg;
    const int lrow0 = l_begin + b * RW;
    const int lm = lrow0 + lane;
    const int lc = (lane < RW && b < nblk && lm < l_end) ? lm : l_begin;
    B.mp = ldg(mu_p + lc);
    B.mm = ldg(mu_m + lc);
    B.fdl = B.fl = B.vp = B.vm = B.sp = B.sm = 0.0;
    if (!prime) {
      B.fdl = ldg(fd + lc);
      B.fl = ldg(flim + lc);
      B.vp = ldg(v_p + lc);
      B.vm = ldg(v_m + lc);
      if (prm.rule != DCOPF_RULE_GDM) {
        B.sp = ldg(s_p + lc);
        B.sm = ldg(s_m + lc);
      }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int lr = (b < nblk && lrow0 + r < l_end) ? lrow0 + r : l_begin;
      const char *row = reinterpret_cast<const char *>(P + (size_t)lr * ldc);
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        B.pr[r][u] = panel_ld<NT>(reinterpret_cast<const V *>(row + cidx[u] * 16u));
    }
  };
  const V *xv = reinterpret_cast<const V *>(x_in);
  V xr[CPL], wacc[CPL];
  const V zero = {};
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    xr[u] = (!prime && cval[u]) ? xv[cidx[u]] : zero;
    wacc[u] = zero;
  }
  const IterSlot cur = sc->slot[par];
  double term = 0.0;
  int it = 0;
  Blk B;
  if (PIPE) load_blk(0, B);
  for (int bb = 0; bb < nblk; bb += NRG, ++it) {
    if (!PIPE) load_blk(bb, B);
    // with PIPE the next block's loads are in flight during this block's work
    Blk Nx;
    const bool more = PIPE && bb + NRG < nblk;
    if (more) load_blk(bb + NRG, Nx);
    const int b = bb + rg;
    const int lm = l_begin + b * RW + lane;
    const bool mine = lane < RW && b < nblk && lm < l_end;
    double dot = 0.0;
    if (!prime) {
      T acc[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        T a = (T)0;
#pragma unroll
        for (int u = 0; u < CPL; ++u) a = fma_vec(B.pr[r][u], xr[u], a);
        acc[r] = wave_sum(a);
      }
      if constexpr (QW > 1) {
        if (lane == 0)
#pragma unroll
          for (int r = 0; r < RW; ++r) dots[it & 1][rg][r][qi] = acc[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          T s = (T)0;
#pragma unroll
          for (int q2 = 0; q2 < QW; ++q2) s += dots[it & 1][rg][r][q2];
          acc[r] = s;
        }
      }
#pragma unroll
      for (int r = 0; r < RW; ++r)
        if (lane == r) dot = (double)acc[r];
    }
    double vnew = 0.0;
    if (mine) {
      const double mp = B.mp, mm = B.mm;
      if (prime) {
        vnew = mp - mm;
      } else {
        double vp = B.vp, vm = B.vm, sp = B.sp, sm = B.sm;
        const double F = dot - B.fdl;
        const double gp = F - B.fl, gm = -F - B.fl;
        const double a = cur.alpha;
        double np_, nm_;
        if (prm.rule == DCOPF_RULE_GDM) {
          vp = prm.rho * vp + a * gp;
          vm = prm.rho * vm + a * gm;
          np_ = mp + vp;
          nm_ = mm + vm;
          if (prm.literal) {
            np_ += a * gp;
            nm_ += a * gm;
          }
        } else if (prm.rule == DCOPF_RULE_ADAM) {
          vp = prm.beta1 * vp + (1.0 - prm.beta1) * gp;
          vm = prm.beta1 * vm + (1.0 - prm.beta1) * gm;
          sp = prm.beta2 * sp + (1.0 - prm.beta2) * gp * gp;
          sm = prm.beta2 * sm + (1.0 - prm.beta2) * gm * gm;
          np_ = mp + a * (vp / cur.c1) / (sqrt(sp / cur.c2) + prm.eps);
          nm_ = mm + a * (vm / cur.c1) / (sqrt(sm / cur.c2) + prm.eps);
        } else {
          sp += gp * gp;
          sm += gm * gm;
          np_ = mp + a * gp / (sqrt(sp) + prm.eps);
          nm_ = mm + a * gm / (sqrt(sm) + prm.eps);
        }
        np_ = fmax(np_, 0.0);
        nm_ = fmax(nm_, 0.0);
        if (qi == 0) {
          term += (mp - mm) * B.fdl + (mp + mm) * B.fl;
          if (prm.rule != DCOPF_RULE_ADAGRAD) {
            v_p[lm] = vp;
            v_m[lm] = vm;
          }
          if (prm.rule != DCOPF_RULE_GDM) {
            s_p[lm] = sp;
            s_m[lm] = sm;
          }
          mu_p[lm] = np_;
          mu_m[lm] = nm_;
        }
        vnew = np_ - nm_;
      }
    }
    // P_l^T v_l of the block's rows, in row order
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const T vr = (T)__shfl(vnew, r, kWave);
#pragma unroll
      for (int u = 0; u < CPL; ++u) wacc[u] = axpy_vec(B.pr[r][u], vr, wacc[u]);
    }
    if (more) B = Nx;
  }
  // one partial of the line terms per workgroup (its wavefronts in order),
  // and the row groups' partials of w meet in LDS: ((W_0 + W_1) + W_2) + W_3
  __shared__ double tw[4];
  if (!prime) {
    const double wl_ = wave_sum(term);
    if (lane == 0) tw[wave] = wl_;
  }
  V *wp = reinterpret_cast<V *>(part_w + (size_t)blockIdx.x * ldc);
  if constexpr (NRG > 1) {
    V *wl = reinterpret_cast<V *>(smem_raw);
    if (rg > 0)
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (cval[u]) wl[(size_t)(rg - 1) * nv + cidx[u]] = wacc[u];
    __syncthreads();
    if (rg == 0)
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (cval[u]) {
          V t = wacc[u];
#pragma unroll
          for (int g = 1; g < NRG; ++g) t += wl[(size_t)(g - 1) * nv + cidx[u]];
          wp[cidx[u]] = t;
        }
  } else {
#pragma unroll
    for (int u = 0; u < CPL; ++u)
      if (cval[u]) wp[cidx[u]] = wacc[u];
    if (!prime) __syncthreads();
  }
  if (!prime && threadIdx.x == 0)
    part_b[(size_t)par * gb + blockIdx.x] = ((tw[0] + tw[1]) + tw[2]) + tw[3];
}

// Units of one column handled by one lane, in unit order (the serial form
// of column_units); the data of the first unit (cf, qf, lof, hif) were
// loaded earlier.
__device__ __forceinline__ void lane_units(double w, double lam, int g0, int g1, double cf,
                                           double qf, double lof, double hif,
                                           const double *__restrict__ c,
                                           const double *__restrict__ q,
                                           const double *__restrict__ pmin,
                                           const double *__restrict__ pmax, double *xj,
                                           double *phij, double *__restrict__ psum, SDual sd,
                                           double alpha, double rho) {
  double xs = 0.0, ph = 0.0;
  for (int t = g0; t < g1; ++t) {
    const bool first = t == g0;
    const double ct = first ? cf : c[t], qt = first ? qf : q[t];
    const double lo = first ? lof : pmin[t], hi = first ? hif : pmax[t];
    const double r = ct - lam + w;
    double p;
    if (sd.s) {
      // Section 3.2, eq. QP_finalgamma with s fixed: q (p - m)^2 is bounded
      // below by -sqrt(q) s (p - m) - s^2 / 4
      const double m = 0.5 * (lo + hi), sq = sqrt(qt), st = sd.s[t];
      const double a = r + 2.0 * qt * m - sq * st;
      p = inner_min(a, 0.0, lo, hi);
      ph += a * p - qt * m * m + sq * st * m - 0.25 * st * st;
      const double v = rho * sd.v[t] + alpha * (-sq * (p - m) - 0.5 * st);
      sd.v[t] = v;
      sd.s[t] = st + v;
    } else {
      p = inner_min(r, qt, lo, hi);
      ph += r * p + qt * p * p;
    }
    xs += p;
    if (psum) psum[t] += p;
  }
  *xj = xs;
  *phij = ph;
}

// Unit pass of the read-once iteration k.  Workgroup j owns the UC columns
// UC j .. UC j + UC - 1 (kUnitCols = UC, 16 or 64); thread (r, c) = (t / UC,
// t % UC) loads the partials g = r, r + 256 / UC, ... (MP of them at most)
// of column UC j + c, all before its first wait, and sums them in FP64 in
// that order; the row sums of a column meet in LDS in row order.
// Wavefront 0 folds iteration k-1 (as the column pass does), then its lanes
// c < UC run the units of column UC j + c and write x; lane 0 writes the
// workgroup's sums of p* and phi.  Every workgroup repeats the fold, whose
// partials grow with the number of workgroups: wide panels take 64 columns
// per workgroup, narrow ones 16 (more workgroups in flight).
template <typename T, int MP, int kUnitCols>
__global__ __launch_bounds__(256) void runits_kernel(
    const T *__restrict__ part_w, int gw, int ldc, int n_cols, const int *__restrict__ seg,
    const double *__restrict__ c, const double *__restrict__ q,
    const double *__restrict__ pmin, const double *__restrict__ pmax, DevScalars *sc, int par,
    T *__restrict__ x_out, double *__restrict__ part_a, int ga,
    const double *__restrict__ part_b, int gb, StepParams prm, double *__restrict__ gam_buf,
    long long gam_mask, double *__restrict__ psum, SDual sd) {
  constexpr int NR = 256 / kUnitCols;
  __shared__ double wr[NR][kUnitCols];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int tc = threadIdx.x % kUnitCols, tr = threadIdx.x / kUnitCols;
  const int col = blockIdx.x * kUnitCols + tc;
  const int cc = col < n_cols ? col : 0;
  const IterSlot prev = sc->slot[par ^ 1];
  const double *pa = part_a + (size_t)(par ^ 1) * 2 * ga;
  const double *pb = part_b + (size_t)(par ^ 1) * gb;
  // wavefront 0: unit boundaries of its column and the previous partials
  const bool ulane = wave == 0 && lane < kUnitCols && col < n_cols;
  int g0 = 0, g1 = 0;
  WaveSums ws;
  if (wave == 0) {
    g0 = ldg(seg + cc);
    g1 = ulane ? ldg(seg + cc + 1) : g0;
    ws.load(pa, ga, pb, gb, lane);
  }
  T pv[MP];
#pragma unroll
  for (int m = 0; m < MP; ++m) {
    const int g = tr + m * NR;
    pv[m] = ldg(part_w + (size_t)(g < gw ? g : 0) * ldc + cc);
  }
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < MP; ++m)
    if (tr + m * NR < gw) s += (double)pv[m];
  // the data of the column's first unit (waits for the boundaries only)
  double cf = 0.0, qf = 0.0, lof = 0.0, hif = 0.0;
  if (wave == 0) {
    const int tf = g0 < g1 ? g0 : 0;
    cf = ldg(c + tf);
    qf = ldg(q + tf);
    lof = ldg(pmin + tf);
    hif = ldg(pmax + tf);
  }
  wr[tr][tc] = s;
  __syncthreads();
  if (wave != 0) return;
  double w = 0.0;
  if (lane < kUnitCols)
#pragma unroll
    for (int r = 0; r < NR; ++r) w += wr[r][lane];
  IterSlot cur = prev;
  if (prev.pending) {
    double ps, phis, lines, gam;
    ws.sum(pa, ga, pb, gb, lane, &ps, &phis, &lines);
    cur = fold(prev, ps, phis, lines, sc->D, prm, &gam);
    if (blockIdx.x == 0 && lane == 0) {
      gam_buf[prev.k & gam_mask] = gam;
      sc->gamma_last = gam;
    }
  }
  set_step(cur, prev.k + 1, prm);
  cur.pending = 1;
  const bool avg = sc->avg_on;
  if (blockIdx.x == 0 && lane == 0) {
    sc->slot[par] = cur;
    if (avg) sc->avg_count += 1;
  }
  double xj = 0.0, phj = 0.0;
  lane_units(w, cur.lam, g0, g1, cf, qf, lof, hif, c, q, pmin, pmax, &xj, &phj,
             avg ? psum : nullptr, sd, cur.alpha, prm.rho);
  if (ulane) x_out[col] = (T)xj;
  const double xs = wave_sum(xj), phs = wave_sum(phj);
  if (lane == 0) {
    part_a[(size_t)par * 2 * ga + 2 * blockIdx.x] = xs;
    part_a[(size_t)par * 2 * ga + 2 * blockIdx.x + 1] = phs;
  }
}

// ---------------------------------------------------------------------------
// Primal recovery (not in the paper): the average pbar of the inner
// minimisers summed by the column passes, its cost and its residuals, in
// FP64.  Columns: pbar per unit, xbar per column (the averaged injection),
// block partials of the cost and of the generation.  Lines: F = P xbar - f_d
// (thread per line, from P^T), block partials of the largest overload, the
// sum of overloads and their count.  A single-thread kernel combines them
// in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kPrimalBlocks = 256;

__global__ __launch_bounds__(256) void primal_cols_kernel(
    const double *__restrict__ psum, const DevScalars *sc, const int *__restrict__ seg,
    const double *__restrict__ c, const double *__restrict__ q, int n_cols,
    double *__restrict__ pbar, double *__restrict__ xbar, double *__restrict__ part) {
  __shared__ double red[2 * 4];
  const double n = (double)sc->avg_count;
  double v[2] = {0.0, 0.0};  // cost, generation
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_cols; j += gridDim.x * blockDim.x) {
    double xs = 0.0;
    for (int u = seg[j]; u < seg[j + 1]; ++u) {
      const double p = psum[u] / n;
      pbar[u] = p;
      v[0] += c[u] * p + q[u] * p * p;
      xs += p;
    }
    xbar[j] = xs;
    v[1] += xs;
  }
  block_sums<2>(v, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = v[0];
    part[gridDim.x + blockIdx.x] = v[1];
  }
}

__global__ __launch_bounds__(256) void primal_lines_kernel(
    const double *__restrict__ P64T, int ldl, int n_cols, int n_lines,
    const double *__restrict__ xbar, const double *__restrict__ fd,
    const double *__restrict__ flim, double *__restrict__ part, double *__restrict__ Fout) {
  __shared__ double red[2 * 4];
  __shared__ double mx_s[4];
  double mx = 0.0, v[2] = {0.0, 0.0};  // sum of overloads, count
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n_lines; l += gridDim.x * blockDim.x) {
    double F = 0.0;
    for (int j = 0; j < n_cols; ++j) F += P64T[(size_t)j * ldl + l] * xbar[j];
    F -= fd[l];
    if (Fout) Fout[l] = F;
    const double o1 = fmax(F - flim[l], 0.0), o2 = fmax(-F - flim[l], 0.0);
    mx = fmax(mx, fmax(o1, o2));
    v[0] += o1 + o2;
    v[1] += (o1 > 0.0 ? 1.0 : 0.0) + (o2 > 0.0 ? 1.0 : 0.0);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
  if (threadIdx.x % kWave == 0) mx_s[threadIdx.x / kWave] = mx;
  block_sums<2>(v, red);  // its barriers also publish mx_s
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) m = fmax(m, mx_s[w]);
    part[blockIdx.x] = m;
    part[gridDim.x + blockIdx.x] = v[0];
    part[2 * gridDim.x + blockIdx.x] = v[1];
  }
}

__global__ void primal_final_kernel(const double *__restrict__ pc, int gc,
                                    const double *__restrict__ pl, int gl, const DevScalars *sc,
                                    DevPrimal *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double cost = 0.0, gen = 0.0, mx = 0.0, sum = 0.0, cnt = 0.0;
  for (int b = 0; b < gc; ++b) {
    cost += pc[b];
    gen += pc[gc + b];
  }
  for (int b = 0; b < gl; ++b) {
    mx = fmax(mx, pl[b]);
    sum += pl[gl + b];
    cnt += pl[2 * gl + b];
  }
  DevPrimal r;
  r.cost = cost;
  r.balance = sc->D - gen;
  r.max_overload = mx;
  r.sum_overload = sum;
  r.count = sc->avg_count;
  r.n_overloaded = (int)cnt;
  r.pad = 0;
  *out = r;
}

// ---------------------------------------------------------------------------
// Repair of a primal candidate into a feasible dispatch (not in the paper).
// One round: units -> column sums x and weights W (FP64), F = P x - f_d per
// line from P^T (primal_lines_kernel), then one workgroup appends the
// violated line directions to the active set in line order and forms the
// targets; the Gram matrix of the active rows and the balance row under the
// weights (one wavefront per entry), its Cholesky factorisation and solve
// in one workgroup, and the step of every unit, clipped to its box.  A unit's
// row value is its column's, so the Gram entries are sums over columns of
// W_c a_ic a_jc with W_c the sum of the column's unit weights.
// ---------------------------------------------------------------------------
constexpr int kRepRows = 256;          // active lines + the balance row
constexpr double kRepMargin = 1e-6;    // MW inside each held limit
constexpr double kRepBalTol = 1e-9;    // of max(1, 1^T d)
constexpr double kRepFloor = 1e-3;     // weight floor, of a unit's range
constexpr double kRepRidge = 1e-12;    // of the largest Gram diagonal

struct RepairState {
  double beta;   // 1^T d - 1^T p of the evaluated iterate
  int n_viol;    // violated line directions
  int m_old, m;  // active lines before / after this evaluation
  int overflow;  // more than kRepRows - 1 lines would be active
  int done;      // stop rule met
  int fail;      // the Gram matrix was not positive definite
};

struct DevRepair {
  double cost, balance, max_overload, max_shift;
};

__device__ __forceinline__ double rep_weight(double p, double lo, double hi) {
  return fmax(fmin(p - lo, hi - p), kRepFloor * (hi - lo));
}

// p = p0c = clip(p0); every line outside the active set; empty set.
__global__ void repair_init_kernel(const double *__restrict__ p0, const double *__restrict__ lo,
                                   const double *__restrict__ hi, int n_gen, int n_lines,
                                   double *__restrict__ p, double *__restrict__ p0c,
                                   int *__restrict__ pos, RepairState *st) {
  const int n = max(n_gen, n_lines);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (i < n_gen) {
      const double v = fmin(fmax(p0[i], lo[i]), hi[i]);
      p[i] = v;
      p0c[i] = v;
    }
    if (i < n_lines) pos[i] = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    RepairState s{};
    *st = s;
  }
}

__global__ __launch_bounds__(256) void repair_cols_kernel(
    const double *__restrict__ p, const int *__restrict__ seg, const double *__restrict__ c,
    const double *__restrict__ q, const double *__restrict__ lo, const double *__restrict__ hi,
    int n_cols, double *__restrict__ x, double *__restrict__ W, double *__restrict__ part) {
  __shared__ double red[2 * 4];
  double v[2] = {0.0, 0.0};  // cost, generation
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_cols; j += gridDim.x * blockDim.x) {
    double xs = 0.0, ws = 0.0;
    for (int u = seg[j]; u < seg[j + 1]; ++u) {
      const double pu = p[u];
      v[0] += c[u] * pu + q[u] * pu * pu;
      xs += pu;
      ws += rep_weight(pu, lo[u], hi[u]);
    }
    x[j] = xs;
    W[j] = ws;
    v[1] += xs;
  }
  block_sums<2>(v, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = v[0];
    part[gridDim.x + blockIdx.x] = v[1];
  }
}

// One workgroup of 256: violations, ordered append to the active set (rows,
// sgn; pos[l] = row of line l or -1), targets t[0..m] (t[m]: balance).
__global__ __launch_bounds__(256) void repair_active_kernel(
    const double *__restrict__ F, const double *__restrict__ flim, int n_lines,
    const double *__restrict__ pcols, int gc, const DevScalars *sc, int *__restrict__ pos,
    int *__restrict__ rows, int *__restrict__ sgn, double *__restrict__ t, RepairState *st) {
  __shared__ int wave_new[4];
  __shared__ int m_s, viol_s, over_s, fail_s;
  __shared__ double beta_s;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  if (tid == 0) {
    double gen = 0.0;
    for (int b = 0; b < gc; ++b) gen += pcols[gc + b];
    beta_s = sc->D - gen;
    m_s = st->m;
    viol_s = 0;
    over_s = st->overflow;
    fail_s = st->fail;
  }
  __syncthreads();
  const int m_old = m_s;
  for (int base = 0; base < n_lines; base += 256) {
    const int l = base + tid;
    int sigma = 0;
    if (l < n_lines) {
      const double Fl = F[l];
      if (Fl - flim[l] > 0.0)
        sigma = 1;
      else if (-Fl - flim[l] > 0.0)
        sigma = -1;
    }
    bool fresh = false;
    if (sigma != 0) {
      const int r = pos[l];
      if (r >= 0)
        sgn[r] = sigma;  // held line: keep its row, take this direction
      else
        fresh = true;
    }
    const unsigned long long mask = __ballot(fresh);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wave_new[wave] = __popcll(mask);
    const int nviol = __popcll(__ballot(sigma != 0));
    __syncthreads();
    int off = m_s;
    for (int w = 0; w < wave; ++w) off += wave_new[w];
    if (fresh) {
      const int r = off + before;
      if (r < kRepRows - 1) {
        rows[r] = l;
        sgn[r] = sigma;
        pos[l] = r;
      }
    }
    __syncthreads();
    if (tid == 0) {
      int add = 0;
      for (int w = 0; w < 4; ++w) add += wave_new[w];
      m_s += add;
    }
    if (lane == 0) atomicAdd(&viol_s, nviol);
    __syncthreads();
  }
  int m = m_s;
  const bool over = m > kRepRows - 1;
  if (over) m = kRepRows - 1;
  for (int i = tid; i < m; i += blockDim.x) {
    const int l = rows[i];
    const double Fl = F[l];
    // flow change that leaves the row kRepMargin inside its limit
    t[i] = sgn[i] > 0 ? (-kRepMargin - (Fl - flim[l])) : (kRepMargin + (-Fl - flim[l]));
  }
  if (tid == 0) {
    t[m] = beta_s;
    RepairState s;
    s.beta = beta_s;
    s.n_viol = viol_s;
    s.m_old = m_old;
    s.m = m;
    s.overflow = (over || over_s) ? 1 : 0;
    s.done = (viol_s == 0 && fabs(beta_s) <= kRepBalTol * fmax(1.0, fabs(sc->D))) ? 1 : 0;
    s.fail = fail_s;
    *st = s;
  }
}

// A[i][c] = P[rows[i]][c] for the rows that joined, zero beyond n_cols.
__global__ void repair_gather_kernel(const double *__restrict__ P64T, int ldl, int n_cols,
                                     int ldc, const int *__restrict__ rows, int m_old,
                                     double *__restrict__ A) {
  const int i = m_old + blockIdx.y;
  const int l = rows[i];
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ldc; j += gridDim.x * blockDim.x)
    A[(size_t)i * ldc + j] = j < n_cols ? P64T[(size_t)j * ldl + l] : 0.0;
}

// G[i][j] (i >= j, n = m + 1 rows; row m is the balance row of ones):
// one wavefront per entry, entries in row-major order of the lower triangle.
__global__ __launch_bounds__(256) void repair_gram_kernel(const double *__restrict__ A, int ldc,
                                                          const double *__restrict__ W,
                                                          int n_cols, int m,
                                                          double *__restrict__ G) {
  const int n = m + 1;
  const long long k = (long long)blockIdx.x * 4 + threadIdx.x / kWave;
  if (k >= (long long)n * (n + 1) / 2) return;
  int i = (int)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
  while ((long long)(i + 1) * (i + 2) / 2 <= k) ++i;
  while ((long long)i * (i + 1) / 2 > k) --i;
  const int j = (int)(k - (long long)i * (i + 1) / 2);
  const int lane = threadIdx.x % kWave;
  const double *ai = A + (size_t)i * ldc, *aj = A + (size_t)j * ldc;
  double s = 0.0;
  for (int c = lane; c < n_cols; c += kWave) {
    const double a = i < m ? ai[c] : 1.0, b = j < m ? aj[c] : 1.0;
    s += W[c] * a * b;
  }
  s = wave_sum(s);
  if (lane == 0) G[(size_t)i * kRepRows + j] = s;
}

// One workgroup: the working-set solve of the step (ws_solve: active lines
// as inequalities, Cholesky in FP64).  st->fail when a pivot is not positive.
__global__ __launch_bounds__(1024) void repair_solve_kernel(const double *__restrict__ G, int m,
                                                            const double *__restrict__ t,
                                                            const int *__restrict__ sgn,
                                                            double *__restrict__ L,
                                                            double *__restrict__ y,
                                                            RepairState *st) {
  __shared__ WsShared sh;
  const bool ok = ws_solve<kRepRows>(G, t, sgn, m, L, y, kRepMargin, kRepRidge, sh);
  if (!ok && threadIdx.x == 0) st->fail = 1;
}

// p_u += w_u z_c (z_c = sum_i y_i A[i][c] + y_m), clipped to the box.
__global__ __launch_bounds__(256) void repair_step_kernel(
    const double *__restrict__ A, int ldc, const double *__restrict__ y, int m,
    const int *__restrict__ seg, const double *__restrict__ lo, const double *__restrict__ hi,
    int n_cols, const RepairState *st, double *__restrict__ p) {
  if (st->fail) return;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_cols; j += gridDim.x * blockDim.x) {
    double z = 0.0;
    for (int i = 0; i < m; ++i) z += y[i] * A[(size_t)i * ldc + j];
    z += y[m];
    for (int u = seg[j]; u < seg[j + 1]; ++u) {
      const double pu = p[u];
      p[u] = fmin(fmax(pu + rep_weight(pu, lo[u], hi[u]) * z, lo[u]), hi[u]);
    }
  }
}

// One workgroup: cost, balance, largest overload and largest shift.
__global__ __launch_bounds__(256) void repair_final_kernel(
    const double *__restrict__ pc, int gc, const double *__restrict__ pl, int gl,
    const DevScalars *sc, const double *__restrict__ p, const double *__restrict__ p0c,
    int n_gen, DevRepair *out) {
  __shared__ double mx_s[4];
  double sh = 0.0;
  for (int u = threadIdx.x; u < n_gen; u += blockDim.x) sh = fmax(sh, fabs(p[u] - p0c[u]));
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) sh = fmax(sh, __shfl_xor(sh, off, kWave));
  if (threadIdx.x % kWave == 0) mx_s[threadIdx.x / kWave] = sh;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double cost = 0.0, gen = 0.0, mo = 0.0, shift = 0.0;
  for (int b = 0; b < gc; ++b) {
    cost += pc[b];
    gen += pc[gc + b];
  }
  for (int b = 0; b < gl; ++b) mo = fmax(mo, pl[b]);
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) shift = fmax(shift, mx_s[w]);
  DevRepair r;
  r.cost = cost;
  r.balance = sc->D - gen;
  r.max_overload = mo;
  r.max_shift = shift;
  *out = r;
}

// Exact bound, column part (FP64): sum over units of phi at the multipliers
// (lambda from `lam`, v = mu+ - mu- in vvec), plus lambda D; last workgroup
// finishes.
template <bool STAGE>
__global__ __launch_bounds__(256) void bound_col_kernel(
    const double *__restrict__ PT, int n_cols, int ldl, const double *__restrict__ vvec,
    const int *__restrict__ seg, const double *__restrict__ c,
    const double *__restrict__ q, const double *__restrict__ pmin,
    const double *__restrict__ pmax, DevScalars *sc, int par, double *__restrict__ part,
    unsigned *counter) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  __shared__ bool last_flag;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const double lam = sc->slot[par].lam;
  const double *vs = vvec;
  if (STAGE) {
    stage_vec(reinterpret_cast<double *>(smem_raw), vvec, ldl);
    __syncthreads();
    vs = reinterpret_cast<const double *>(smem_raw);
  }
  const int nv = ldl / 2;
  double phisum = 0.0;
  for (int j = blockIdx.x * nw + wave; j < n_cols; j += gridDim.x * nw) {
    const double w = wave_sum(lane_dot<double, true>(PT + (size_t)j * ldl, vs, nv, lane));
    double xj, phij;
    column_units(j, w, lam, seg, c, q, pmin, pmax, lane, &xj, &phij);
    if (lane == 0) phisum += phij;
  }
  const double bphi = block_sum(phisum, red);
  if (threadIdx.x == 0) store_agent(part + blockIdx.x, bphi);
  if (!last_block_done(counter, &last_flag)) return;
  double t = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) t += load_agent(part + b);
  t = block_sum(t, red);
  if (threadIdx.x == 0) sc->bound_gen = t + lam * sc->D;
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
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) t += load_agent(part + b);
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

template <typename T> T *dalloc(DevPool &pool, size_t n, dcopf_status *st) {
  T *p = pool.get_n<T>(n == 0 ? 1 : n);
  if (!p) *st = DCOPF_E_NOMEM;
  return p;
}

bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

struct dcopf_dual_s {
  DevPool pool;  // every device buffer of the handle (the caller's allocator)
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
  std::vector<int> gperm_h;  // host copy: unit t of the column order is generator gperm_h[t]
  // state
  double *mu_p = nullptr, *mu_m = nullptr, *v_p = nullptr, *v_m = nullptr, *s_p = nullptr,
         *s_m = nullptr;
  void *vbuf = nullptr, *xbuf = nullptr;  // loop precision vectors (padded)
  double *v64b = nullptr;                 // FP64 v for the exact bound
  double *part_a = nullptr, *part_b = nullptr;  // iteration partials [2][...] by parity
  double *part_c = nullptr, *part_d = nullptr;  // exact-bound partials
  unsigned *counters = nullptr;
  DevScalars *sc = nullptr;
  double *gam = nullptr;
  // primal average: sum of p* per unit (column order), evaluation buffers
  double *psum = nullptr, *pbar = nullptr, *xbar = nullptr, *ppart = nullptr;
  DevPrimal *primal = nullptr;
  // the iterated-s QP dual: s and its velocity per unit (column order)
  double *s_unit = nullptr, *v_unit = nullptr;
  // primal repair (allocated by its first call)
  struct Repair {
    double *pin = nullptr, *p = nullptr, *p0c = nullptr, *x = nullptr, *W = nullptr,
           *F = nullptr, *t = nullptr, *y = nullptr, *G = nullptr, *L = nullptr, *A = nullptr,
           *pc = nullptr, *pl = nullptr;
    int *pos = nullptr, *rows = nullptr, *sgn = nullptr;
    RepairState *st = nullptr;
    DevRepair *out = nullptr;
    bool ready = false;
  } rep;
  // launch shapes
  int grid_col = 0, grid_line = 0, grid_bnd_col = 0, grid_bnd_line = 0;
  int n_line_part = 0;  // line-pass partials: one per wavefront
  size_t lds_col = 0, lds_line = 0, lds_bnd = 0;
  bool stage_col = false, stage_line = false, stage_bnd = false;
  int col_cb = 1;   // panel columns per workgroup in the column pass
  bool col_one = false;  // one-column, one-barrier column pass (small panels)
  bool panel_nt = false;  // panels too large for the last-level cache: nontemporal loads
  int line_xr = 0;  // x chunks per lane held in registers (0: LDS / global)
  // read-once iteration (line pass forms the next w's partials; unit pass)
  bool fused = false;
  int rl_qw = 1, rl_rw = 4, rl_cpl = 1, grid_rl = 0, grid_units = 0, unit_cols = 16;
  size_t lds_rl = 0;
  void *part_w = nullptr;  // [grid_rl][ldc] in the loop precision
  // graph of graph_iters iterations (even), starting at an even iteration
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_iters = 0;
  // host bookkeeping
  long long iters = 0;
  double best = -INFINITY;
  long long best_iter = -1;
  double cost_ub = INFINITY;  // largest possible generation cost
};

namespace {

constexpr int kLineRows = 4;  // lines per wavefront in the line pass

// Workgroups per compute unit the read-once line pass aims at (the
// partials of w it writes grow with the count)
#ifndef DCOPF_READ_ONCE_GROUPS_PER_CU
#define DCOPF_READ_ONCE_GROUPS_PER_CU 2
#endif
constexpr int kReadOnceGroupsPerCU = DCOPF_READ_ONCE_GROUPS_PER_CU;
// The next block's panel loads issued before the current block's work
#ifndef DCOPF_READ_ONCE_PIPE
#define DCOPF_READ_ONCE_PIPE 0
#endif
constexpr bool kReadOncePipe = DCOPF_READ_ONCE_PIPE != 0;
// Rows per wavefront and block when a row has at most 2 chunks per lane
#ifndef DCOPF_ROWS_NARROW
#define DCOPF_ROWS_NARROW 4
#endif
constexpr int kRowsNarrow = DCOPF_ROWS_NARROW;
// Rows of up to this many chunks per lane are covered by one wavefront
#ifndef DCOPF_QW1_MAX_CPL
#define DCOPF_QW1_MAX_CPL 12
#endif
constexpr int kQw1MaxCpl = DCOPF_QW1_MAX_CPL;
// Automatic scheme: panels below this size (loop precision) keep the
// two-pass iteration (measured: a 6 MB panel iterates faster two-pass, a
// 21 MB one read-once)
#ifndef DCOPF_READ_ONCE_MIN_BYTES
#define DCOPF_READ_ONCE_MIN_BYTES (10 << 20)
#endif
constexpr double kReadOnceMinBytes = DCOPF_READ_ONCE_MIN_BYTES;
// Panels wider than this many columns are "wide" for the read-once layout
constexpr int kWideUnitCols = 4096;
static_assert(kQw1MaxCpl == 4 || kQw1MaxCpl == 12, "one-wavefront rows: 4 or 12 chunks");

template <typename T, int CB, int UNR>
void launch_colpass_cb(dcopf_dual_s *h, hipStream_t s, int par, hipEvent_t e0, hipEvent_t e1) {
  T *PT = std::is_same<T, float>::value ? (T *)h->P32T : (T *)h->P64T;
  (void)launch_k(h->panel_nt ? colpass_kernel<T, CB, UNR, true> : colpass_kernel<T, CB, UNR, false>,
                 dim3(h->grid_col), dim3(256), 0, s, e0, e1, PT,
                 h->n_cols, h->ldl, (T *)h->vbuf, h->seg, h->c, h->q, h->pmin, h->pmax, h->sc,
                 par, (T *)h->xbuf, h->part_a, h->grid_col, h->part_b, h->n_line_part, h->prm,
                 h->gam, kGamCap - 1, h->psum, SDual{h->s_unit, h->v_unit});
}

template <typename T, int UNR>
void launch_colpass1(dcopf_dual_s *h, hipStream_t s, int par, hipEvent_t e0, hipEvent_t e1) {
  T *PT = std::is_same<T, float>::value ? (T *)h->P32T : (T *)h->P64T;
  (void)launch_k(colpass1_kernel<T, UNR>, dim3(h->grid_col), dim3(256), 0, s, e0, e1, PT,
                 h->n_cols, h->ldl, (T *)h->vbuf, h->seg, h->c, h->q, h->pmin, h->pmax, h->sc,
                 par, (T *)h->xbuf, h->part_a, h->grid_col, h->part_b, h->n_line_part, h->prm,
                 h->gam, kGamCap - 1, h->psum, SDual{h->s_unit, h->v_unit});
}

// one column per workgroup and a quarter of at most 8 chunks per lane: the
// one-barrier column pass; otherwise the general one
template <typename T>
void launch_colpass(dcopf_dual_s *h, hipStream_t s, int par, hipEvent_t e0, hipEvent_t e1) {
  const int quarter = (h->ldl / Vec16<T>::n + 3) / 4;
  if (h->col_one) {
    if (quarter <= 4 * kWave) launch_colpass1<T, 4>(h, s, par, e0, e1);
    else launch_colpass1<T, 8>(h, s, par, e0, e1);
  } else if (h->col_cb == 1) {
    launch_colpass_cb<T, 1, 0>(h, s, par, e0, e1);
  } else if (h->col_cb == 2) {
    launch_colpass_cb<T, 2, 0>(h, s, par, e0, e1);
  } else {
    launch_colpass_cb<T, 4, 0>(h, s, par, e0, e1);
  }
}

template <typename T>
void launch_linepass(dcopf_dual_s *h, hipStream_t s, int par, hipEvent_t e0, hipEvent_t e1) {
  T *P = std::is_same<T, float>::value ? (T *)h->P32 : (T *)h->P64;
  T *v = (T *)h->vbuf, *x = (T *)h->xbuf;
#define DCOPF_LINEPASS(STAGE, XR, NT, LDS)                                                   \
  (void)launch_k(linepass_kernel<T, STAGE, kLineRows, XR, NT>, dim3(h->grid_line), dim3(256),  \
                 LDS,                                                                          \
                 s, e0, e1, P, h->n_lines, h->ldc, x, h->fd, h->fmax, h->mu_p, h->mu_m,       \
                 h->v_p, h->v_m, h->s_p, h->s_m, v, h->sc, par, h->part_b, h->n_line_part, h->prm)
  // x in registers (narrow panels): plain loads
  if (h->line_xr == 2) DCOPF_LINEPASS(false, 2, false, 0);
  else if (h->line_xr == 4) DCOPF_LINEPASS(false, 4, false, 0);
  else if (h->stage_line && h->panel_nt) DCOPF_LINEPASS(true, 0, true, (unsigned)h->lds_line);
  else if (h->stage_line) DCOPF_LINEPASS(true, 0, false, (unsigned)h->lds_line);
  else if (h->panel_nt) DCOPF_LINEPASS(false, 0, true, 0);
  else DCOPF_LINEPASS(false, 0, false, 0);
#undef DCOPF_LINEPASS
}

template <typename T, int QW, int RW, int CPL>
void launch_rlines_cfg(dcopf_dual_s *h, hipStream_t s, int par, int prime, hipEvent_t e0,
                       hipEvent_t e1) {
  T *P = std::is_same<T, float>::value ? (T *)h->P32 : (T *)h->P64;
  constexpr bool PIPE = kReadOncePipe && QW > 1;
  (void)launch_k(h->panel_nt ? rlines_kernel<T, QW, RW, CPL, true, PIPE>
                             : rlines_kernel<T, QW, RW, CPL, false, PIPE>,
                 dim3(h->grid_rl), dim3(256), (unsigned)h->lds_rl, s, e0, e1, P, h->n_lines,
                 h->ldc, (T *)h->xbuf, h->fd, h->fmax, h->mu_p, h->mu_m, h->v_p, h->v_m,
                 h->s_p, h->s_m, h->sc, par, h->part_b, h->n_line_part, (T *)h->part_w, h->prm,
                 prime);
}

template <typename T>
void launch_rlines(dcopf_dual_s *h, hipStream_t s, int par, int prime, hipEvent_t e0 = nullptr,
                   hipEvent_t e1 = nullptr) {
  if (h->rl_qw == 1) {
    switch (h->rl_cpl) {
      case 1: launch_rlines_cfg<T, 1, kRowsNarrow, 1>(h, s, par, prime, e0, e1); break;
      case 2: launch_rlines_cfg<T, 1, kRowsNarrow, 2>(h, s, par, prime, e0, e1); break;
      case 4: launch_rlines_cfg<T, 1, 4, 4>(h, s, par, prime, e0, e1); break;
#if DCOPF_QW1_MAX_CPL > 4
      case 6: launch_rlines_cfg<T, 1, 2, 6>(h, s, par, prime, e0, e1); break;
      case 9: launch_rlines_cfg<T, 1, 2, 9>(h, s, par, prime, e0, e1); break;
      default: launch_rlines_cfg<T, 1, 2, 12>(h, s, par, prime, e0, e1); break;
#else
      default: break;
#endif
    }
    return;
  }
  // rows per block: about 24 chunks per lane in flight (twice that, in two
  // blocks, when the next block's loads go out before this block's work)
  constexpr int D = kReadOncePipe ? 2 : 1;
  switch (h->rl_cpl) {
    case 2: launch_rlines_cfg<T, 4, 8 / D, 2>(h, s, par, prime, e0, e1); break;
    case 3: launch_rlines_cfg<T, 4, 8 / D, 3>(h, s, par, prime, e0, e1); break;
    case 4: launch_rlines_cfg<T, 4, 8 / D, 4>(h, s, par, prime, e0, e1); break;
    case 6: launch_rlines_cfg<T, 4, 4 / D, 6>(h, s, par, prime, e0, e1); break;
    case 8: launch_rlines_cfg<T, 4, 4 / D, 8>(h, s, par, prime, e0, e1); break;
    case 10: launch_rlines_cfg<T, 4, 2 / D, 10>(h, s, par, prime, e0, e1); break;
    case 12: launch_rlines_cfg<T, 4, 2 / D, 12>(h, s, par, prime, e0, e1); break;
    default: launch_rlines_cfg<T, 4, 2 / D, 16>(h, s, par, prime, e0, e1); break;
  }
}

template <typename T, int MP, int UC>
void launch_runits_mp(dcopf_dual_s *h, hipStream_t s, int par, hipEvent_t e0, hipEvent_t e1) {
  (void)launch_k(runits_kernel<T, MP, UC>, dim3(h->grid_units), dim3(256), 0, s, e0, e1,
                 (T *)h->part_w, h->grid_rl, h->ldc, h->n_cols, h->seg, h->c, h->q, h->pmin,
                 h->pmax, h->sc, par, (T *)h->xbuf, h->part_a, h->grid_units, h->part_b,
                 h->n_line_part, h->prm, h->gam, kGamCap - 1, h->psum,
                 SDual{h->s_unit, h->v_unit});
}

// partials per thread: at most 16 MP line-pass workgroups
template <typename T, int UC>
void launch_runits_uc(dcopf_dual_s *h, hipStream_t s, int par, hipEvent_t e0, hipEvent_t e1) {
  constexpr int NR = 256 / UC;
  if (h->grid_rl <= NR * 4) launch_runits_mp<T, 4, UC>(h, s, par, e0, e1);
  else if (h->grid_rl <= NR * 8) launch_runits_mp<T, 8, UC>(h, s, par, e0, e1);
  else if (h->grid_rl <= NR * 16) launch_runits_mp<T, 16, UC>(h, s, par, e0, e1);
  else if (h->grid_rl <= NR * 32) launch_runits_mp<T, 32, UC>(h, s, par, e0, e1);
  else launch_runits_mp<T, 64, UC>(h, s, par, e0, e1);
}

template <typename T>
void launch_runits(dcopf_dual_s *h, hipStream_t s, int par, hipEvent_t e0, hipEvent_t e1) {
  if (h->unit_cols == 16) launch_runits_uc<T, 16>(h, s, par, e0, e1);
  else launch_runits_uc<T, 64>(h, s, par, e0, e1);
}

// Partials of w = P^T v for the current multipliers (after create or a set
// state), so the next unit pass starts from them.
void prime_w(dcopf_dual_s *h) {
  if (!h->fused) return;
  if (h->opts.precision == DCOPF_PREC_FP32) launch_rlines<float>(h, h->stream, 0, 1);
  else launch_rlines<double>(h, h->stream, 0, 1);
}

void launch_phase(dcopf_dual_s *h, hipStream_t s, int phase, int par, hipEvent_t e0 = nullptr,
                  hipEvent_t e1 = nullptr) {
  const bool fp32 = h->opts.precision == DCOPF_PREC_FP32;
  if (h->fused) {
    if (phase == 0) {
      if (fp32) launch_runits<float>(h, s, par, e0, e1);
      else launch_runits<double>(h, s, par, e0, e1);
    } else {
      if (fp32) launch_rlines<float>(h, s, par, 0, e0, e1);
      else launch_rlines<double>(h, s, par, 0, e0, e1);
    }
    return;
  }
  if (phase == 0) {
    if (fp32) launch_colpass<float>(h, s, par, e0, e1);
    else launch_colpass<double>(h, s, par, e0, e1);
  } else {
    if (fp32) launch_linepass<float>(h, s, par, e0, e1);
    else launch_linepass<double>(h, s, par, e0, e1);
  }
}

// n iterations starting at iteration index `first` (parity from the index)
void launch_iters(dcopf_dual_s *h, hipStream_t s, long long first, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    const int par = (int)((first + i) & 1);
    launch_phase(h, s, 0, par);
    launch_phase(h, s, 1, par);
  }
}

// Fold the partials of the last launched iteration (no-op when none pending).
void launch_finalize(dcopf_dual_s *h, hipStream_t s) {
  const int par = (int)((h->iters - 1) & 1);
  finalize_kernel<<<1, 256, 0, s>>>(h->sc, par, h->part_a,
                                    h->fused ? h->grid_units : h->grid_col, h->part_b,
                                    h->n_line_part, h->prm, h->gam, kGamCap - 1,
                                    (h->fused || h->col_one) ? 1 : 0);
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

// Host copy of the scalars; the folded state of iteration iters - 1.
dcopf_status read_scalars(dcopf_dual_s *h, DevScalars *out) {
  DCOPF_HIP_TRY(hipStreamSynchronize(h->stream));
  DCOPF_HIP_TRY(hipMemcpy(out, h->sc, sizeof(DevScalars), hipMemcpyDeviceToHost));
  return DCOPF_OK;
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
  if (nl > (1u << 20) || nb > (1u << 24))
    return set_error("at most 2^20 lines and 2^24 buses"), DCOPF_E_INVALID;
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
  if (o->qp_dual != DCOPF_QP_CLOSED && o->qp_dual != DCOPF_QP_ITERATED)
    return set_error("unknown qp_dual"), DCOPF_E_INVALID;
  if (o->scheme < DCOPF_SCHEME_AUTO || o->scheme > DCOPF_SCHEME_READ_ONCE)
    return set_error("unknown scheme"), DCOPF_E_INVALID;
  if (o->qp_dual == DCOPF_QP_ITERATED &&
      (o->rule != DCOPF_RULE_GDM || o->literal != 0 || o->decay != 0.0))
    return set_error("the iterated-s QP dual needs rule GDM, literal 0, decay 0"),
           DCOPF_E_INVALID;
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
  h->pool.release_all();
  delete h;
}

int grid_for(int rows, int rows_per_block, int max_blocks) {
  int g = (rows + rows_per_block - 1) / rows_per_block;
  return std::max(1, std::min(g, max_blocks));
}

}  // namespace

extern "C" {

const char *dcopf_last_error(void) { return get_error(); }

dcopf_status dcopf_set_allocator(dcopf_alloc_fn alloc, dcopf_free_fn free, void *ctx) {
  if ((alloc == nullptr) != (free == nullptr))
    return set_error("set_allocator: give both functions or neither"), DCOPF_E_INVALID;
  g_mem = DevMem{alloc, free, alloc ? ctx : nullptr, nullptr};
  return DCOPF_OK;
}

dcopf_status dcopf_dual_create(const dcopf_problem *p, const dcopf_opts *o, void *hip_stream,
                               dcopf_dual_t *out) {
  if (!out) return set_error("out is NULL"), DCOPF_E_INVALID;
  *out = nullptr;
  set_error("");
  dcopf_status st = validate(p, o);
  if (st != DCOPF_OK) return st;
  auto *h = new dcopf_dual_s();
  h->stream = (hipStream_t)hip_stream;
  h->pool.mem = current_devmem(hip_stream);
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
  h->panel_nt = ((size_t)nl * h->ldc + (size_t)nc * h->ldl) * esz > kMallBytes;

  // launch shapes: 4 wavefronts per workgroup
  // column pass: enough workgroups to cover the chip (one to four columns
  // each); line pass: x in registers when a row has at most 4 chunks per lane
  h->col_cb = nc >= 2048 ? 4 : (nc >= 1024 ? 2 : 1);
  h->grid_col = (nc + h->col_cb - 1) / h->col_cb;
  {
    const int per_chunk = o->precision == DCOPF_PREC_FP32 ? 4 : 2;
    const int quarter = (h->ldl / per_chunk + 3) / 4;
    h->col_one = h->col_cb == 1 && quarter <= 8 * kWave;
  }
  {
    const int nvc = h->ldc / (fp32 ? 4 : 2);
    h->line_xr = nvc <= 128 ? 2 : (nvc <= 256 ? 4 : 0);
  }
  h->grid_line = grid_for(nl, 4 * kLineRows, 65536);
  h->n_line_part = 4 * h->grid_line;
  {
    // read-once iteration: rows of up to 4 chunks per lane are covered by
    // one wavefront (four row groups per workgroup), wider rows by the four
    // wavefronts together (up to 16 chunks per lane); wider panels keep the
    // two-pass iteration
    const int nvc = h->ldc / (fp32 ? 4 : 2);
    int qw = 1, cpl = (nvc + kWave - 1) / kWave;
    if (cpl > kQw1MaxCpl) {
      qw = 4;
      cpl = (nvc + 4 * kWave - 1) / (4 * kWave);
    }
    static const int kCpl1[] = {1, 2, 4, 4, 6, 6, 9, 9, 9, 12, 12, 12},
                     kCpl4[] = {2, 3, 4, 6, 8, 10, 12, 16};
    if (qw == 1) cpl = kCpl1[cpl - 1];
    else
      for (int v : kCpl4)
        if (v >= cpl) {
          cpl = v;
          break;
        }
    const bool can = qw == 1 || cpl <= 16;
    if (o->scheme == DCOPF_SCHEME_READ_ONCE && !can) {
      free_handle(h);
      return set_error("read-once scheme: panel rows too wide (use two-pass)"), DCOPF_E_INVALID;
    }
    h->fused = o->scheme == DCOPF_SCHEME_READ_ONCE ||
               (o->scheme == DCOPF_SCHEME_AUTO && can &&
                (double)nl * h->ldc * (fp32 ? 4 : 8) >= (double)kReadOnceMinBytes);
    if (h->fused) {
      h->rl_qw = qw;
      h->rl_cpl = cpl;
      h->rl_rw = qw == 1 ? (cpl <= 2 ? kRowsNarrow : (cpl <= 4 ? 4 : 2))
                         : (cpl <= 4 ? 8 : (cpl <= 8 ? 4 : 2)) / (kReadOncePipe ? 2 : 1);
      // workgroups: one block round each while that keeps the count below
      // the target (a few per compute unit), else the target
      const int rows_m = h->rl_rw * (4 / qw);
      int n_cu = 256;
      {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            v > 0)
          n_cu = v;
      }
      // wide panels: 64 columns per unit-pass workgroup and one line-pass
      // workgroup per compute unit (half the partials); narrow ones: 16
      // columns and two per compute unit
      const bool wide = nc > kWideUnitCols;
      h->unit_cols = wide ? 64 : 16;
      const int target = std::max(1, (wide ? 1 : kReadOnceGroupsPerCU) * n_cu);
      h->grid_rl = std::min(target, (nl + rows_m - 1) / rows_m);
      h->grid_rl = std::max(1, std::min(h->grid_rl, nl));
      h->grid_rl = std::min(h->grid_rl, (256 / h->unit_cols) * 64);  // the unit pass's limit
      h->lds_rl = (size_t)(4 / qw - 1) * h->ldc * (fp32 ? 4 : 8);
      h->n_line_part = h->grid_rl;
      h->grid_units = (nc + h->unit_cols - 1) / h->unit_cols;
      h->panel_nt = (size_t)nl * h->ldc * (fp32 ? 4 : 8) > kMallBytes;
    }
  }
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
    h->P32 = dalloc<float>(h->pool, panel, &st);
    if (!h->fused) h->P32T = dalloc<float>(h->pool, panelT, &st);
  } else {
    h->P64 = dalloc<double>(h->pool, panel, &st);
  }
  h->P64T = dalloc<double>(h->pool, panelT, &st);
  h->fd = dalloc<double>(h->pool, nl, &st);
  h->fmax = dalloc<double>(h->pool, nl, &st);
  h->c = dalloc<double>(h->pool, ng, &st);
  h->q = dalloc<double>(h->pool, ng, &st);
  h->pmin = dalloc<double>(h->pool, ng, &st);
  h->pmax = dalloc<double>(h->pool, ng, &st);
  h->seg = dalloc<int>(h->pool, nc + 1, &st);
  h->gperm = dalloc<int>(h->pool, ng, &st);
  double **state[] = {&h->mu_p, &h->mu_m, &h->v_p, &h->v_m, &h->s_p, &h->s_m};
  for (double **s : state) *s = dalloc<double>(h->pool, nl, &st);
  h->vbuf = dalloc<unsigned char>(h->pool, (size_t)h->ldl * esz, &st);
  h->xbuf = dalloc<unsigned char>(h->pool, (size_t)h->ldc * esz, &st);
  h->v64b = dalloc<double>(h->pool, h->ldl, &st);
  h->part_a = dalloc<double>(h->pool, 4 * (size_t)std::max(h->grid_col, h->grid_units), &st);
  if (h->fused) h->part_w = dalloc<unsigned char>(h->pool, (size_t)h->grid_rl * h->ldc * esz, &st);
  h->part_b = dalloc<double>(h->pool, 2 * (size_t)h->n_line_part, &st);
  h->part_c = dalloc<double>(h->pool, (size_t)h->grid_bnd_line, &st);
  h->part_d = dalloc<double>(h->pool, (size_t)h->grid_bnd_col, &st);
  h->counters = dalloc<unsigned>(h->pool, 8, &st);
  h->sc = dalloc<DevScalars>(h->pool, 1, &st);
  h->psum = dalloc<double>(h->pool, ng, &st);
  if (o->qp_dual == DCOPF_QP_ITERATED) {
    h->s_unit = dalloc<double>(h->pool, ng, &st);
    h->v_unit = dalloc<double>(h->pool, ng, &st);
  }
  h->pbar = dalloc<double>(h->pool, ng, &st);
  h->xbar = dalloc<double>(h->pool, (size_t)h->n_cols, &st);
  h->ppart = dalloc<double>(h->pool, 5 * (size_t)kPrimalBlocks, &st);  // column and line partials
  h->primal = dalloc<DevPrimal>(h->pool, 1, &st);
  h->gam = dalloc<double>(h->pool, kGamCap, &st);
  double *Hd = nullptr, *dd = nullptr;
  int *dcols = nullptr;
  Hd = dalloc<double>(h->pool, (size_t)nl * nb, &st);
  dd = dalloc<double>(h->pool, nb, &st);
  dcols = dalloc<int>(h->pool, nc, &st);
  auto cleanup_tmp = [&]() {
    h->pool.put(Hd);
    h->pool.put(dd);
    h->pool.put(dcols);
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
  // unit data in column-sorted order (unit t of the panel = generator gperm[t])
  std::vector<double> cs(ng), qs(ng, 0.0), lo(ng), hi(ng);
  for (int t = 0; t < ng; ++t) {
    const int g = gperm[t];
    cs[t] = p->c[g];
    qs[t] = p->q ? p->q[g] : 0.0;
    lo[t] = p->p_min[g];
    hi[t] = p->p_max[g];
  }
  chk(hipMemcpyAsync(h->c, cs.data(), ng * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->q, qs.data(), ng * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->pmin, lo.data(), ng * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->pmax, hi.data(), ng * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->fmax, p->f_max, nl * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->seg, seg.data(), (nc + 1) * 4, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(h->gperm, gperm.data(), ng * 4, hipMemcpyHostToDevice, s));
  h->gperm_h = gperm;
  for (double **sp : state) chk(hipMemsetAsync(*sp, 0, nl * 8, s));
  if (h->s_unit) {
    chk(hipMemsetAsync(h->s_unit, 0, (size_t)ng * 8, s));
    chk(hipMemsetAsync(h->v_unit, 0, (size_t)ng * 8, s));
  }
  chk(hipMemsetAsync(h->xbuf, 0, (size_t)h->ldc * esz, s));
  chk(hipMemsetAsync(h->counters, 0, 8 * sizeof(unsigned), s));
  chk(hipMemsetAsync(h->gam, 0, kGamCap * 8, s));
  DevScalars sch{};
  double D = 0.0;
  for (int b = 0; b < nb; ++b) D += p->d[b];
  sch.D = D;
  // cold start (Algorithm 1): lambda = 0, no iteration done; the slot of
  // iteration -1 (parity 1) is what iteration 0 reads
  sch.slot[1].k = -1;
  sch.slot[0].k = -2;
  chk(hipMemcpyAsync(h->sc, &sch, sizeof(sch), hipMemcpyHostToDevice, s));
  // panels
  {
    dim3 gg((unsigned)std::min<int64_t>(64, (h->ldc + 255) / 256), (unsigned)nl);
    // the transposed panels are written over their full padded width ldl
    dim3 tg((unsigned)(h->ldc / 32), (unsigned)(h->ldl / 32));
    if (fp32) {
      gather_kernel<float><<<gg, 256, 0, s>>>(Hd, nb, nl, dcols, nc, h->ldc, h->P32);
      if (h->P32T)
        transpose_kernel<float><<<tg, dim3(32, 8), 0, s>>>(h->P32, nl, h->ldc, nc, h->ldl, h->P32T);
      // FP64 panel for the bound, transposed: gather into the (free) T slot first
      double *tmp = nullptr;
      tmp = h->pool.get_n<double>(panel);
      if (!tmp) chk(hipErrorOutOfMemory);
      if (tmp) {
        gather_kernel<double><<<gg, 256, 0, s>>>(Hd, nb, nl, dcols, nc, h->ldc, tmp);
        transpose_kernel<double><<<tg, dim3(32, 8), 0, s>>>(tmp, nl, h->ldc, nc, h->ldl, h->P64T);
        chk(hipStreamSynchronize(s));
        h->pool.put(tmp);
      }
    } else {
      gather_kernel<double><<<gg, 256, 0, s>>>(Hd, nb, nl, dcols, nc, h->ldc, h->P64);
      transpose_kernel<double><<<tg, dim3(32, 8), 0, s>>>(h->P64, nl, h->ldc, nc, h->ldl, h->P64T);
    }
    hd_kernel<<<grid_for(nl, 4, 4096), 256, 0, s>>>(Hd, nb, nl, dd, h->fd);
  }
  chk(hipGetLastError());
  refresh_v(h);
  prime_w(h);
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
  // capture graph_iters (rounded up to even) iterations, starting at an even
  // iteration, into a HIP graph (on a private stream)
  h->graph_iters = (o->graph_iters + 1) / 2 * 2;
  if (h->graph_iters > 0) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      free_handle(h);
      return set_error("hipStreamCreate failed"), DCOPF_E_HIP;
    }
    hipError_t ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (ce == hipSuccess) {
      launch_iters(h, cs, 0, h->graph_iters);
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
  if (n == 0) return DCOPF_OK;
  int64_t left = n;
  if (h->graph_exec) {
    if (h->iters & 1) {  // the graph starts at an even iteration
      launch_iters(h, h->stream, h->iters, 1);
      h->iters += 1;
      left -= 1;
    }
    const int gi = h->graph_iters;
    while (left >= gi) {
      DCOPF_HIP_TRY(hipGraphLaunch(h->graph_exec, h->stream));
      h->iters += gi;
      left -= gi;
    }
  }
  launch_iters(h, h->stream, h->iters, left);
  h->iters += left;
  launch_finalize(h, h->stream);
  DCOPF_HIP_TRY(hipGetLastError());
  return DCOPF_OK;
}

static dcopf_status eval_bound(dcopf_dual_t h, double *value) {
  hipStream_t s = h->stream;
  const int blocks = (int)std::min<int64_t>(1024, (h->ldl + 255) / 256);
  const int par = (int)((h->iters - 1) & 1);  // slot holding the current lambda
  make_v_kernel<double><<<blocks, 256, 0, s>>>(h->mu_p, h->mu_m, h->n_lines, h->ldl, h->v64b);
  if (h->stage_bnd)
    bound_col_kernel<true><<<h->grid_bnd_col, 256, h->lds_bnd, s>>>(
        h->P64T, h->n_cols, h->ldl, h->v64b, h->seg, h->c, h->q, h->pmin, h->pmax,
        h->sc, par, h->part_d, h->counters + 2);
  else
    bound_col_kernel<false><<<h->grid_bnd_col, 256, 0, s>>>(
        h->P64T, h->n_cols, h->ldl, h->v64b, h->seg, h->c, h->q, h->pmin, h->pmax,
        h->sc, par, h->part_d, h->counters + 2);
  bound_lines_kernel<<<h->grid_bnd_line, 256, 0, s>>>(h->mu_p, h->mu_m, h->fd, h->fmax,
                                                       h->n_lines, h->sc, h->part_c,
                                                       h->counters + 3);
  DCOPF_HIP_TRY(hipGetLastError());
  DevScalars sch;
  dcopf_status st = read_scalars(h, &sch);
  if (st != DCOPF_OK) return st;
  *value = sch.bound_value;
  if (!std::isfinite(sch.bound_value) || !std::isfinite(sch.slot[par].lam))
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
    dcopf_status s2 = read_scalars(h, &sch);
    if (s2 != DCOPF_OK) return s2;
    *lambda = sch.slot[(h->iters - 1) & 1].lam;
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
  st = read_scalars(h, &sch);
  if (st != DCOPF_OK) return st;
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
  if (h->s_unit) return set_error("not available with the iterated-s QP dual"), DCOPF_E_INVALID;
  if (len != dcopf_dual_state_len(h)) return set_error("state length mismatch"), DCOPF_E_STATE;
  DevScalars sch;
  dcopf_status st = read_scalars(h, &sch);
  if (st != DCOPF_OK) return st;
  const IterSlot &sl = sch.slot[(h->iters - 1) & 1];
  buf[0] = (double)h->iters;
  buf[1] = sl.lam;
  buf[2] = sl.v_lam;
  buf[3] = sl.s_lam;
  buf[4] = 0.0;
  const size_t nl = h->n_lines;
  double *arrs[] = {h->mu_p, h->mu_m, h->v_p, h->v_m, h->s_p, h->s_m};
  for (int i = 0; i < 6; ++i)
    DCOPF_HIP_TRY(hipMemcpy(buf + 5 + i * nl, arrs[i], nl * 8, hipMemcpyDeviceToHost));
  return DCOPF_OK;
}

dcopf_status dcopf_dual_set_state(dcopf_dual_t h, const double *buf, size_t len) {
  if (!h || !buf) return set_error("null argument"), DCOPF_E_INVALID;
  if (h->s_unit) return set_error("not available with the iterated-s QP dual"), DCOPF_E_INVALID;
  if (len != dcopf_dual_state_len(h)) return set_error("state length mismatch"), DCOPF_E_STATE;
  if (!finite_all(buf, len)) return set_error("non-finite state"), DCOPF_E_INVALID;
  const size_t nl = h->n_lines;
  for (size_t i = 0; i < 2 * nl; ++i)
    if (buf[5 + i] < 0.0) return set_error("mu must be >= 0"), DCOPF_E_INVALID;
  if (buf[0] < 0 || buf[0] != std::floor(buf[0]) || buf[0] > 1e15)
    return set_error("iteration must be a nonnegative integer"), DCOPF_E_INVALID;
  DevScalars sch;
  dcopf_status st = read_scalars(h, &sch);
  if (st != DCOPF_OK) return st;
  const long long k0 = (long long)buf[0];
  IterSlot sl{};
  sl.lam = buf[1];
  sl.v_lam = buf[2];
  sl.s_lam = buf[3];
  sl.k = k0 - 1;
  sl.pending = 0;
  sch.slot[(k0 - 1) & 1] = sl;
  sch.slot[k0 & 1] = IterSlot{};
  sch.slot[k0 & 1].k = k0 - 2;
  DCOPF_HIP_TRY(hipMemcpy(h->sc, &sch, sizeof(sch), hipMemcpyHostToDevice));
  double *arrs[] = {h->mu_p, h->mu_m, h->v_p, h->v_m, h->s_p, h->s_m};
  for (int i = 0; i < 6; ++i)
    DCOPF_HIP_TRY(hipMemcpy(arrs[i], buf + 5 + i * nl, nl * 8, hipMemcpyHostToDevice));
  h->iters = k0;
  refresh_v(h);
  prime_w(h);
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(h->stream));
  return DCOPF_OK;
}

dcopf_status dcopf_dual_time_phases(dcopf_dual_t h, int64_t n, double *ms_out) {
  if (!h || !ms_out || n < 1) return set_error("bad arguments"), DCOPF_E_INVALID;
  if (h->s_unit) return set_error("not available with the iterated-s QP dual"), DCOPF_E_INVALID;
  // n real iterations (column pass, line pass alternating as in step), each
  // launch carrying dispatch-attached start/stop events; the mutable state is
  // saved first and restored afterwards, so the iterate is unchanged.
  const size_t nl = h->n_lines;
  const size_t esz = h->opts.precision == DCOPF_PREC_FP32 ? 4 : 8;
  double *save = nullptr;
  void *vsave = nullptr;
  DevScalars *ssave = nullptr;
  // the loop-precision vector the first timed launch reads: v (two-pass
  // iteration) or the partials of w = P^T v (read-once iteration)
  void *vbuf = h->fused ? h->part_w : h->vbuf;
  const size_t vbytes = h->fused ? (size_t)h->grid_rl * h->ldc * esz : (size_t)h->ldl * esz;
  save = h->pool.get_n<double>(6 * nl);
  vsave = h->pool.get(vbytes);
  ssave = h->pool.get_n<DevScalars>(1);
  if (!save || !vsave || !ssave) {
    h->pool.put(save);
    h->pool.put(vsave);
    h->pool.put(ssave);
    return set_error("time_phases: device allocation failed"), DCOPF_E_NOMEM;
  }
  double *arrs[] = {h->mu_p, h->mu_m, h->v_p, h->v_m, h->s_p, h->s_m};
  hipStream_t s = h->stream;
  for (int i = 0; i < 6; ++i)
    DCOPF_HIP_TRY(hipMemcpyAsync(save + i * nl, arrs[i], nl * 8, hipMemcpyDeviceToDevice, s));
  DCOPF_HIP_TRY(hipMemcpyAsync(vsave, vbuf, vbytes, hipMemcpyDeviceToDevice, s));
  DCOPF_HIP_TRY(hipMemcpyAsync(ssave, h->sc, sizeof(DevScalars), hipMemcpyDeviceToDevice, s));
  // the timed iterations add nothing to a primal average in progress
  static const int zero = 0;
  DCOPF_HIP_TRY(hipMemcpyAsync(&h->sc->avg_on, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  std::vector<hipEvent_t> ev(4 * (size_t)n, nullptr);
  for (auto &e : ev) DCOPF_HIP_TRY(hipEventCreate(&e));
  for (int64_t i = 0; i < n; ++i) {
    const int par = (int)((h->iters + i) & 1);
    for (int phase = 0; phase < 2; ++phase)
      launch_phase(h, s, phase, par, ev[4 * i + 2 * phase], ev[4 * i + 2 * phase + 1]);
  }
  for (int i = 0; i < 6; ++i)
    DCOPF_HIP_TRY(hipMemcpyAsync(arrs[i], save + i * nl, nl * 8, hipMemcpyDeviceToDevice, s));
  DCOPF_HIP_TRY(hipMemcpyAsync(vbuf, vsave, vbytes, hipMemcpyDeviceToDevice, s));
  DCOPF_HIP_TRY(hipMemcpyAsync(h->sc, ssave, sizeof(DevScalars), hipMemcpyDeviceToDevice, s));
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(s));
  double acc[2] = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i)
    for (int phase = 0; phase < 2; ++phase) {
      float ms = 0.f;
      DCOPF_HIP_TRY(hipEventElapsedTime(&ms, ev[4 * i + 2 * phase], ev[4 * i + 2 * phase + 1]));
      acc[phase] += ms;
    }
  for (int phase = 0; phase < 2; ++phase) ms_out[phase] = acc[phase] / n;
  for (auto &e : ev) (void)hipEventDestroy(e);
  h->pool.put(save);
  h->pool.put(vsave);
  h->pool.put(ssave);
  return DCOPF_OK;
}

dcopf_status dcopf_dual_average(dcopf_dual_t h, int32_t enable) {
  if (!h) return set_error("null handle"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(h->stream));
  DevScalars sch;
  dcopf_status st = read_scalars(h, &sch);
  if (st != DCOPF_OK) return st;
  if (enable) {
    DCOPF_HIP_TRY(hipMemset(h->psum, 0, (size_t)h->n_gen * 8));
    sch.avg_count = 0;
  }
  sch.avg_on = enable ? 1 : 0;
  DCOPF_HIP_TRY(hipMemcpy(h->sc, &sch, sizeof(sch), hipMemcpyHostToDevice));
  return DCOPF_OK;
}

dcopf_status dcopf_dual_primal(dcopf_dual_t h, dcopf_primal *out, double *p_avg) {
  if (!h || !out) return set_error("null argument"), DCOPF_E_INVALID;
  DevScalars sch;
  dcopf_status st = read_scalars(h, &sch);  // synchronises
  if (st != DCOPF_OK) return st;
  if (sch.avg_count <= 0) return set_error("no iterations averaged"), DCOPF_E_STATE;
  const int gc = std::max(1, std::min(kPrimalBlocks, (h->n_cols + 255) / 256));
  const int gl = std::max(1, std::min(kPrimalBlocks, (h->n_lines + 255) / 256));
  hipStream_t s = h->stream;
  primal_cols_kernel<<<gc, 256, 0, s>>>(h->psum, h->sc, h->seg, h->c, h->q, h->n_cols, h->pbar,
                                        h->xbar, h->ppart);
  primal_lines_kernel<<<gl, 256, 0, s>>>(h->P64T, h->ldl, h->n_cols, h->n_lines, h->xbar, h->fd,
                                         h->fmax, h->ppart + 2 * kPrimalBlocks, nullptr);
  primal_final_kernel<<<1, 64, 0, s>>>(h->ppart, gc, h->ppart + 2 * kPrimalBlocks, gl, h->sc,
                                       h->primal);
  DCOPF_HIP_TRY(hipGetLastError());
  DevPrimal r;
  DCOPF_HIP_TRY(hipMemcpyAsync(&r, h->primal, sizeof(r), hipMemcpyDeviceToHost, s));
  std::vector<double> pb;
  if (p_avg) {
    pb.resize(h->n_gen);
    DCOPF_HIP_TRY(hipMemcpyAsync(pb.data(), h->pbar, pb.size() * 8, hipMemcpyDeviceToHost, s));
  }
  DCOPF_HIP_TRY(hipStreamSynchronize(s));
  out->cost = r.cost;
  out->balance = r.balance;
  out->max_overload = r.max_overload;
  out->sum_overload = r.sum_overload;
  out->iterations = r.count;
  out->n_overloaded = r.n_overloaded;
  if (p_avg)  // unit t of the column order is generator gperm_h[t]
    for (int t = 0; t < h->n_gen; ++t) p_avg[h->gperm_h[t]] = pb[t];
  return DCOPF_OK;
}

dcopf_status dcopf_dual_repair(dcopf_dual_t h, const double *p_in, int32_t max_rounds,
                               dcopf_repair *out, double *p_out) {
  if (!h || !out || max_rounds < 0) return set_error("bad arguments"), DCOPF_E_INVALID;
  const int ng = h->n_gen, nl = h->n_lines, nc = h->n_cols;
  if (p_in && !finite_all(p_in, (size_t)ng)) return set_error("p_in is not finite"), DCOPF_E_INVALID;
  auto &R = h->rep;
  if (!R.ready) {
    dcopf_status st = DCOPF_OK;
    R.pin = dalloc<double>(h->pool, ng, &st);
    R.p = dalloc<double>(h->pool, ng, &st);
    R.p0c = dalloc<double>(h->pool, ng, &st);
    R.x = dalloc<double>(h->pool, nc, &st);
    R.W = dalloc<double>(h->pool, nc, &st);
    R.F = dalloc<double>(h->pool, nl, &st);
    R.t = dalloc<double>(h->pool, kRepRows, &st);
    R.y = dalloc<double>(h->pool, kRepRows, &st);
    R.G = dalloc<double>(h->pool, (size_t)kRepRows * kRepRows, &st);
    R.L = dalloc<double>(h->pool, (size_t)kRepRows * kRepRows, &st);
    R.A = dalloc<double>(h->pool, (size_t)kRepRows * h->ldc, &st);
    R.pc = dalloc<double>(h->pool, 2 * (size_t)kPrimalBlocks, &st);
    R.pl = dalloc<double>(h->pool, 3 * (size_t)kPrimalBlocks, &st);
    R.pos = dalloc<int>(h->pool, nl, &st);
    R.rows = dalloc<int>(h->pool, kRepRows, &st);
    R.sgn = dalloc<int>(h->pool, kRepRows, &st);
    R.st = dalloc<RepairState>(h->pool, 1, &st);
    R.out = dalloc<DevRepair>(h->pool, 1, &st);
    if (st != DCOPF_OK) return set_error("device allocation failed"), st;
    R.ready = true;
  }
  hipStream_t s = h->stream;
  const int gc = std::max(1, std::min(kPrimalBlocks, (nc + 255) / 256));
  const int gl = std::max(1, std::min(kPrimalBlocks, (nl + 255) / 256));
  const double *src = R.pin;
  if (p_in) {
    std::vector<double> pc(ng);  // unit t of the column order is generator gperm_h[t]
    for (int t = 0; t < ng; ++t) pc[t] = p_in[h->gperm_h[t]];
    DCOPF_HIP_TRY(hipMemcpyAsync(R.pin, pc.data(), (size_t)ng * 8, hipMemcpyHostToDevice, s));
    DCOPF_HIP_TRY(hipStreamSynchronize(s));
  } else {
    DevScalars sch;
    dcopf_status st = read_scalars(h, &sch);
    if (st != DCOPF_OK) return st;
    if (sch.avg_count <= 0) return set_error("no iterations averaged"), DCOPF_E_STATE;
    primal_cols_kernel<<<gc, 256, 0, s>>>(h->psum, h->sc, h->seg, h->c, h->q, nc, h->pbar,
                                          h->xbar, h->ppart);
    src = h->pbar;
  }
  const int gi = std::min(1024, (std::max(ng, nl) + 255) / 256);
  repair_init_kernel<<<gi, 256, 0, s>>>(src, h->pmin, h->pmax, ng, nl, R.p, R.p0c, R.pos, R.st);
  const int ldc = h->ldc;
  int rounds = 0;
  RepairState hs{};
  for (;;) {
    repair_cols_kernel<<<gc, 256, 0, s>>>(R.p, h->seg, h->c, h->q, h->pmin, h->pmax, nc, R.x,
                                          R.W, R.pc);
    primal_lines_kernel<<<gl, 256, 0, s>>>(h->P64T, h->ldl, nc, nl, R.x, h->fd, h->fmax, R.pl,
                                           R.F);
    repair_active_kernel<<<1, 256, 0, s>>>(R.F, h->fmax, nl, R.pc, gc, h->sc, R.pos, R.rows,
                                           R.sgn, R.t, R.st);
    DCOPF_HIP_TRY(hipGetLastError());
    DCOPF_HIP_TRY(hipMemcpyAsync(&hs, R.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    DCOPF_HIP_TRY(hipStreamSynchronize(s));
    if (hs.done || hs.fail || hs.overflow || rounds >= max_rounds) break;
    if (hs.m > hs.m_old) {
      dim3 gg((unsigned)((ldc + 255) / 256), (unsigned)(hs.m - hs.m_old));
      repair_gather_kernel<<<gg, 256, 0, s>>>(h->P64T, h->ldl, nc, ldc, R.rows, hs.m_old, R.A);
    }
    const long long pairs = (long long)(hs.m + 1) * (hs.m + 2) / 2;
    repair_gram_kernel<<<(unsigned)((pairs + 3) / 4), 256, 0, s>>>(R.A, ldc, R.W, nc, hs.m, R.G);
    repair_solve_kernel<<<1, 1024, 0, s>>>(R.G, hs.m, R.t, R.sgn, R.L, R.y, R.st);
    repair_step_kernel<<<(nc + 255) / 256, 256, 0, s>>>(R.A, ldc, R.y, hs.m, h->seg, h->pmin,
                                                        h->pmax, nc, R.st, R.p);
    ++rounds;
  }
  if (hs.fail) --rounds;  // the failed solve moved nothing
  repair_final_kernel<<<1, 256, 0, s>>>(R.pc, gc, R.pl, gl, h->sc, R.p, R.p0c, ng, R.out);
  DCOPF_HIP_TRY(hipGetLastError());
  DevRepair r;
  DCOPF_HIP_TRY(hipMemcpyAsync(&r, R.out, sizeof(r), hipMemcpyDeviceToHost, s));
  std::vector<double> pb;
  if (p_out) {
    pb.resize(ng);
    DCOPF_HIP_TRY(hipMemcpyAsync(pb.data(), R.p, (size_t)ng * 8, hipMemcpyDeviceToHost, s));
  }
  DCOPF_HIP_TRY(hipStreamSynchronize(s));
  out->cost = r.cost;
  out->balance = r.balance;
  out->max_overload = r.max_overload;
  out->max_shift = r.max_shift;
  out->feasible = hs.done ? 1 : 0;
  out->rounds = rounds;
  out->n_active = hs.m;
  out->pad = 0;
  if (p_out)
    for (int t = 0; t < ng; ++t) p_out[h->gperm_h[t]] = pb[t];
  return DCOPF_OK;
}

dcopf_status dcopf_dual_info(dcopf_dual_t h, int32_t *n_cols, int64_t *iters) {
  if (!h) return set_error("null handle"), DCOPF_E_INVALID;
  if (n_cols) *n_cols = h->n_cols;
  if (iters) *iters = h->iters;
  return DCOPF_OK;
}

dcopf_status dcopf_dual_scheme(dcopf_dual_t h, int32_t *scheme, int32_t *line_groups) {
  if (!h) return set_error("null handle"), DCOPF_E_INVALID;
  if (scheme) *scheme = h->fused ? DCOPF_SCHEME_READ_ONCE : DCOPF_SCHEME_TWO_PASS;
  if (line_groups) *line_groups = h->fused ? h->grid_rl : 0;
  return DCOPF_OK;
}

void dcopf_dual_destroy(dcopf_dual_t h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  free_handle(h);
}

}  // extern "C"
