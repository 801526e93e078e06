// Batched projected dual ascent (many DCOPF instances) on CDNA4 matrix cores.
//
// Instances of one network share its generator-bus panel P (lines x columns)
// and differ in loads d_i (hence f_d,i = H d_i) and costs c_i, q_i.  With the
// instances as the M dimension, one iteration (Section 3.3, Algorithm 1 and
// its variants, run for every instance) is three launches, each covering
// every network through a tile table:
//
//   W product   W^T = V^T P   (M = instances, N = panel columns, K = lines)
//               split-BF16 v_mfma_f32_32x32x16_bf16, FP32 accumulation,
//               optional split over K for long-K / few-instance networks;
//               workgroups after the tiles fold the previous iteration: the
//               lambda step with its balance residual (FP64) and its monitor
//               value gamma;
//   unit pass   one workgroup per instance and 512 columns: w = sum of the
//               K splits, reduced costs r = c - lambda + w (FP64), the
//               closed-form inner minimiser (Sections 3.1 / 3.2), the
//               column injections X (written as BF16 hi/lo), sum p* and
//               sum phi;
//   F product   F^T = X^T P^T (M = instances, N = lines, K = columns), whose
//               epilogue forms F - f_d, the residuals +-F - f_max, the mu
//               step and projection (FP32 state), the next V (BF16 hi/lo) and
//               the line terms of gamma.
//
// Every operand is read with K contiguous (16-byte loads per lane) and every
// state array is written coalesced along the N index of the output tile.
// The exact bound uses FP64 products on v_mfma_f64_16x16x4f64.
#include "common.h"
#include "../../include/dcopf_batch.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace dcopf {
namespace {

struct BNet {
  int n_l, n_c, n_g, B, Bp, ldl, ldc, ncp, nlp, S, kchunk, inst0, ntl;
  int cfg_w, cfg_f;  // workgroup tile shape codes of the W and F products
  int nt_panel;      // panel operands read nontemporally (a panel too large to stay cached)
  double alpha, rho;
  const __bf16 *PT_hi, *PT_lo, *P_hi, *P_lo;
  const double *P64T;
  __bf16 *V_hi, *V_lo, *X_hi, *X_lo;
  float *Wws;                                   // [S][Bp][ncp]
  float *mu_p, *mu_m, *v_p, *v_m, *s_p, *s_m;   // [B][ldl]
  const float *fd32;                            // [B][ldl]
  const float *flim32;                          // [n_l]
  const double *flim64, *fd64;                  // [n_l], [B][n_l]
  const double *c, *q;                          // [B][n_g]
  const double *pmin, *pmax;                    // [n_g]
  const int *seg;                               // units of column j: seg[j] .. seg[j+1]-1
                                                // (unit data stored column-sorted)
  const int *ucol;                              // [n_g]: column of each unit
  double *lam, *vlam, *slam;                    // [2][B]: state used by the iteration of that parity
  double *D;                                    // [B]
  int ncb;                                      // column blocks of the unit pass
  double *unitpart;                             // [2][ncb][Bp][2]: sum p*, sum phi by parity
  double *linepart;                             // [ntl][Bp]
  double *V64, *W64;                            // [Bp][ldl], [Bp][ncp]
  double *bound;                                // [B]
  // primal average (an extension): sum of p* per instance and unit
  // (column-sorted), the FP64 panel [lines][ldc] for F = P xbar, buffers
  double *psum;                                 // [B][n_g]
  double *P64;                                  // [nlp][ldc]
  double *X64, *F64;                            // [Bp][ldc], [Bp][nlp]
  double *pbar;                                 // [B][n_g]
  double *ppart;                                // [B][5]: cost, generation, max, sum, count
};

struct BIter {
  long long k;  // iteration index of this slot
  int pending;  // gamma of iteration k - 1 not yet finished
  int pad;
};

struct BScal {
  BIter it[2];
  long long avg_count;  // iterations summed into the primal average
  int avg_on, avg_pad;  // unit passes add p* to the primal sums
};

struct BParams {
  int rule, literal;
  double beta1, beta2, eps, decay;
};

__device__ __forceinline__ double inner_min_b(double r, double q, double lo, double hi) {
  if (q > 0.0) return fmin(fmax(-r / (2.0 * q), lo), hi);
  if (r > 0.0) return lo;
  if (r < 0.0) return hi;
  return 0.5 * (lo + hi);
}

__device__ __forceinline__ void split_bf16(float v, __bf16 *hi, __bf16 *lo) {
  const __bf16 h = (__bf16)v;
  *hi = h;
  *lo = (__bf16)(v - (float)h);
}

// Output element of v_mfma_f32_32x32x16: register j of lane l holds row
// 8 (j / 4) + 4 (l / 32) + j % 4 and column l % 32.
__device__ __forceinline__ int mfma32_row(int j, int lane) {
  return 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
}

// element at a 32-bit byte offset (per-network state arrays are < 4 GiB)
// (loads and stores through global-address-space pointers)
template <typename T> __device__ __forceinline__ T ld_at(const T *p, unsigned byte_off) {
  return ldg(reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + byte_off));
}
template <typename T> __device__ __forceinline__ void st_at(T *p, unsigned byte_off, T v) {
  *(__attribute__((address_space(1))) T *)(reinterpret_cast<char *>(p) + byte_off) = v;
}

// largest K split of the W product (the unit pass holds every split's
// partial of its column in registers)
constexpr int kMaxSplit = 32;

// Split panels (hi and lo, both orientations) of at least this many bytes
// are read nontemporally
#ifndef DCOPF_BATCH_NT_PANEL_BYTES
#define DCOPF_BATCH_NT_PANEL_BYTES (128.0 * 1024 * 1024)
#endif
constexpr double kNtPanelBytes = DCOPF_BATCH_NT_PANEL_BYTES;

// ---------------------------------------------------------------------------
// Workgroup tile of a split-BF16 product, staged through LDS.
//
// C[BM x BN] += (A_hi + A_lo)[BM x K] (B_hi + B_lo)[BN x K]^T over k in
// [kb, ke) (a multiple of 64).  256 threads = WM x WN wavefronts, each owning
// TM x TN tiles of 32 x 32 (v_mfma_f32_32x32x16_bf16).  Per 64-deep K step the
// four operand tiles are copied to LDS (8 threads per 128-byte row) from one
// of two register stages, that stage is refilled with the loads of the step
// after next before the products, and the fragments are read from LDS with a
// 144-byte row stride (16-byte reads of 16 consecutive rows hit disjoint
// banks).
// ---------------------------------------------------------------------------
constexpr int kBK = 64;
constexpr int kLdsStride = kBK + 8;  // bf16 elements per LDS row

template <int BM, int BN> struct TileLds {
  __bf16 a[2][BM][kLdsStride];
  __bf16 b[2][BN][kLdsStride];
};

template <int BM, int BN, int WM, int WN, bool LOLO>
__device__ __forceinline__ void tile_mma(const __bf16 *__restrict__ Ah,
                                         const __bf16 *__restrict__ Al, int lda,
                                         const __bf16 *__restrict__ Bh,
                                         const __bf16 *__restrict__ Bl, int ldb, int kb, int ke,
                                         TileLds<BM, BN> &sm,
                                         f32x16 (&acc)[BM / (WM * 32)][BN / (WN * 32)],
                                         bool nt_b) {
  constexpr int TM = BM / (WM * 32), TN = BN / (WN * 32);
  constexpr int RA = BM / 32, RB = BN / 32;  // 32-row groups per operand tile
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int lrow = t >> 3, lchunk = (t & 7) * 8;
  // two register stages: while step k is copied to LDS and multiplied, the
  // loads of steps k + 1 and k + 2 are in flight
  bf16x8 pa0[2][RA], pb0[2][RB], pa1[2][RA], pb1[2][RB];
  auto fetch = [&](bf16x8 (&pa)[2][RA], bf16x8 (&pb)[2][RB], int k) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const size_t off = (size_t)(r * 32 + lrow) * lda + k + lchunk;
      pa[0][r] = ldg(reinterpret_cast<const bf16x8 *>(Ah + off));
      pa[1][r] = ldg(reinterpret_cast<const bf16x8 *>(Al + off));
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const size_t off = (size_t)(r * 32 + lrow) * ldb + k + lchunk;
      if (nt_b) {
        pb[0][r] = __builtin_nontemporal_load(reinterpret_cast<const bf16x8 *>(Bh + off));
        pb[1][r] = __builtin_nontemporal_load(reinterpret_cast<const bf16x8 *>(Bl + off));
      } else {
        pb[0][r] = ldg(reinterpret_cast<const bf16x8 *>(Bh + off));
        pb[1][r] = ldg(reinterpret_cast<const bf16x8 *>(Bl + off));
      }
    }
  };
  const int fr = lane & 31, fk = (lane >> 5) * 8;
  auto step = [&](bf16x8 (&pa)[2][RA], bf16x8 (&pb)[2][RB], int k) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int r = 0; r < RA; ++r)
        *reinterpret_cast<bf16x8 *>(&sm.a[h][r * 32 + lrow][lchunk]) = pa[h][r];
#pragma unroll
      for (int r = 0; r < RB; ++r)
        *reinterpret_cast<bf16x8 *>(&sm.b[h][r * 32 + lrow][lchunk]) = pb[h][r];
    }
    __syncthreads();
    // refill this stage with the step after next (clamped to the last step:
    // the loads stay unconditional, so each wait counts exactly the loads
    // still needed)
    fetch(pa, pb, min(k + 2 * kBK, ke - kBK));
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
      bf16x8 fa[2][TM], fb[2][TN];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
          fa[h][i] = *reinterpret_cast<const bf16x8 *>(
              &sm.a[h][(wm * TM + i) * 32 + fr][kk + fk]);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          fb[h][j] = *reinterpret_cast<const bf16x8 *>(
              &sm.b[h][(wn * TN + j) * 32 + fr][kk + fk]);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0][i], fb[0][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0][i], fb[1][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1][i], fb[0][j], acc[i][j], 0, 0, 0);
          if (LOLO)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1][i], fb[1][j], acc[i][j], 0, 0, 0);
        }
    }
  };
  if (kb >= ke) return;
  fetch(pa0, pb0, kb);
  fetch(pa1, pb1, min(kb + kBK, ke - kBK));
  int k = kb;
  for (; k + 2 * kBK <= ke; k += 2 * kBK) {
    step(pa0, pb0, k);
    step(pa1, pb1, k + kBK);
  }
  if (k < ke) step(pa0, pb0, k);  // odd number of K steps
}

// Workgroup tile shapes (code stored per network): BM x BN and wave layout.
//   0: 128 x 64 (2 x 2 waves, 64 x 32 each)   1: 64 x 128 (2 x 2, 32 x 64)
//   2: 32 x 128 (1 x 4, 32 x 32)
#define DCOPF_TILE_SWITCH(code, BODY)                                                      \
  switch (code) {                                                                         \
    case 0: { BODY(128, 64, 2, 2); } break;                                               \
    case 1: { BODY(64, 128, 2, 2); } break;                                               \
    default: { BODY(32, 128, 1, 4); } break;                                              \
  }

constexpr int kTileBM[3] = {128, 64, 32};
constexpr int kTileBN[3] = {64, 128, 128};
// one LDS buffer serves every shape (the largest is 128 + 64 rows)
constexpr int kTileLdsBytes = (int)sizeof(TileLds<128, 64>);
static_assert(sizeof(TileLds<64, 128>) <= (size_t)kTileLdsBytes, "LDS");
static_assert(sizeof(TileLds<32, 128>) <= (size_t)kTileLdsBytes, "LDS");

// ---------------------------------------------------------------------------
// W product: Wws[s][i][j] = sum_{l in split s} V[i][l] P[l][j]
// ---------------------------------------------------------------------------
template <int BM, int BN, int WM, int WN, bool LOLO>
__device__ __forceinline__ void wgemm_body(const BNet &N, int4 t, unsigned char *lds) {
  constexpr int TM = BM / (WM * 32), TN = BN / (WN * 32);
  TileLds<BM, BN> &sm = *reinterpret_cast<TileLds<BM, BN> *>(lds);
  const int m0 = t.y * BM, n0 = t.z * BN;
  const int kb = t.w * N.kchunk, ke = min(N.ldl, kb + N.kchunk);
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  tile_mma<BM, BN, WM, WN, LOLO>(N.V_hi + (size_t)m0 * N.ldl, N.V_lo + (size_t)m0 * N.ldl,
                                 N.ldl, N.PT_hi + (size_t)n0 * N.ldl,
                                 N.PT_lo + (size_t)n0 * N.ldl, N.ldl, kb, ke, sm, acc,
                                 N.nt_panel != 0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int mb = m0 + (wm * TM + i) * 32, n = n0 + (wn * TN + j) * 32 + (lane & 31);
      float *out = N.Wws + ((size_t)t.w * N.Bp + mb) * N.ncp + n;
#pragma unroll
      for (int e = 0; e < 16; ++e) out[(size_t)mfma32_row(e, lane) * N.ncp] = acc[i][j][e];
    }
}


// The state (lambda, velocity or first moment, second moment) of iteration
// k from that of iteration k-1 (slot pp) and its sums f = (sum p*, sum phi,
// line terms), and the dual value gamma of iteration k-1.
struct LamState {
  double lam, v, s, gamma;
};

__device__ __forceinline__ LamState fold_finish(const BNet &N, int i, int pp, long long k_prev,
                                                const BParams &prm, const double (&f)[3]) {
  const double lam = N.lam[(size_t)pp * N.B + i];
  const double v0 = N.vlam[(size_t)pp * N.B + i], s0 = N.slam[(size_t)pp * N.B + i];
  const double D = N.D[i];
  LamState r;
  r.gamma = f[1] + lam * D - f[2];
  const double kk = (double)k_prev;
  const double a = (prm.decay == 0.0 ? N.alpha : N.alpha / (1.0 + prm.decay * kk));
  const double g = D - f[0];  // balance residual
  r.v = v0;
  r.s = s0;
  if (prm.rule == DCOPF_RULE_GDM) {
    r.v = N.rho * v0 + a * g;
    r.lam = lam + r.v + (prm.literal ? a * g : 0.0);
  } else if (prm.rule == DCOPF_RULE_ADAM) {
    const double c1 = 1.0 - pow(prm.beta1, kk + 1.0), c2 = 1.0 - pow(prm.beta2, kk + 1.0);
    r.v = prm.beta1 * v0 + (1.0 - prm.beta1) * g;
    r.s = prm.beta2 * s0 + (1.0 - prm.beta2) * g * g;
    r.lam = lam + a * (r.v / c1) / (sqrt(r.s / c2) + prm.eps);
  } else {
    r.s = s0 + g * g;
    r.lam = lam + a * g / (sqrt(r.s) + prm.eps);
  }
  return r;
}

// Fold of iteration k-1 (parity pp) of instance i by one wavefront: the
// lanes stride over the partial sums that iteration left (the unit pass's
// sums of p* and phi per column block, the F product's line terms per 32-line
// tile), a butterfly over the wavefront adds them up (every lane ends with
// the same sums, in a fixed order), then lambda's state for iteration k goes
// to slot pp ^ 1 and gamma of iteration k-1 to the ring.
__device__ __forceinline__ void fold_wave(const BNet &N, int i, int pp, long long k_prev,
                                          const BParams &prm, double *__restrict__ gam_ring,
                                          long long gmask, int n_total) {
  const int lane = threadIdx.x & 63;
  double f[3] = {0.0, 0.0, 0.0};
  const double *up = N.unitpart + (size_t)pp * N.ncb * N.Bp * 2;
  for (int t = lane; t < N.ncb; t += 64) {
    f[0] += ldg(up + ((size_t)t * N.Bp + i) * 2);
    f[1] += ldg(up + ((size_t)t * N.Bp + i) * 2 + 1);
  }
  for (int t = lane; t < N.ntl; t += 64) f[2] += ldg(N.linepart + (size_t)t * N.Bp + i);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int v = 0; v < 3; ++v) f[v] += __shfl_xor(f[v], o, 64);
  const LamState r = fold_finish(N, i, pp, k_prev, prm, f);
  if (lane == 0) {
    const int np = pp ^ 1;
    N.lam[(size_t)np * N.B + i] = r.lam;
    N.vlam[(size_t)np * N.B + i] = r.v;
    N.slam[(size_t)np * N.B + i] = r.s;
    gam_ring[(size_t)(k_prev & gmask) * n_total + N.inst0 + i] = r.gamma;
  }
}

// Workgroups 0 .. n_tiles-1: the W product's tiles.  The ones after them
// (dispatched last, so they fill the tail of the launch) fold iteration k-1
// of four instances each, one per wavefront, so that the unit pass of
// iteration k finds lambda ready.
template <bool LOLO>
__global__ __launch_bounds__(256) void wgemm_kernel(const BNet *__restrict__ nets,
                                                    const int4 *__restrict__ tiles, int n_tiles,
                                                    const int2 *__restrict__ inst_tab,
                                                    const BScal *sc, int par, BParams prm,
                                                    double *__restrict__ gam_ring,
                                                    long long gmask, int n_total) {
  __shared__ __align__(16) unsigned char lds[kTileLdsBytes];
  if ((int)blockIdx.x >= n_tiles) {
    const BIter it = sc->it[par];
    const int slot = ((int)blockIdx.x - n_tiles) * 4 + (int)(threadIdx.x >> 6);
    if (it.pending && slot < n_total) {
      const int2 e = inst_tab[slot];
      fold_wave(nets[e.x], e.y, par ^ 1, it.k - 1, prm, gam_ring, gmask, n_total);
    }
    return;
  }
  const int4 t = tiles[blockIdx.x];
  const BNet &N = nets[t.x];
#define DCOPF_WBODY(BM, BN, WM, WN) wgemm_body<BM, BN, WM, WN, LOLO>(N, t, lds)
  DCOPF_TILE_SWITCH(N.cfg_w, DCOPF_WBODY)
#undef DCOPF_WBODY
}

// ---------------------------------------------------------------------------
// Unit pass: workgroup (instance i, column block cb) handles the columns
// jb = cb kUnitCols .. je - 1, kUnitCPT per thread (columns jb + t and
// jb + t + 256), and their units ub .. ue - 1 (unit data are stored
// column-sorted, so a block's units are contiguous; the workgroup's entry of
// the unit table carries ub and ue, so no unit load waits for a boundary
// lookup).  Every load that does
// not depend on lambda is issued first: for the thread's columns the K-split
// partials of w and the unit boundaries, for its units (one per thread and
// round, consecutive threads on consecutive units) their data and column.
// Lambda of this iteration was folded in the W launch.  Then w of every
// column goes to LDS; the units are evaluated (reduced cost, inner
// minimiser, phi) into LDS, kUnitChunk at a time; each column adds its
// units' p* and phi in unit order; the injections X (BF16 hi/lo) and the
// workgroup's sums of p* and phi are stored.  MAXS bounds the K split.
// ---------------------------------------------------------------------------
constexpr int kUnitCPT = 2;
constexpr int kUnitCols = 256 * kUnitCPT;
constexpr int kUnitRounds = 3;  // units per thread and chunk
constexpr int kUnitChunk = 256 * kUnitRounds;

template <int MAXS>
__global__ __launch_bounds__(256) void units_kernel(const BNet *__restrict__ nets,
                                                    const int4 *__restrict__ unit_tab,
                                                    BScal *sc, int par) {
  __shared__ double wcol[kUnitCols];
  __shared__ double pch[kUnitChunk], phch[kUnitChunk];
  __shared__ double red[2 * 4];
  const int4 e = unit_tab[blockIdx.x];
  const BNet &N = nets[e.x & 0xffff];
  const int i = e.y, cb = e.x >> 16, ub = e.z, ue = e.w;
  const int jb = cb * kUnitCols, je = min(N.n_c, jb + kUnitCols);
  // loads are issued unconditionally from clamped (in-range) indices and
  // masked afterwards, so that none of them waits for another
  int jj[kUnitCPT], u0[kUnitCPT], u1[kUnitCPT];
  bool valid[kUnitCPT];
#pragma unroll
  for (int h = 0; h < kUnitCPT; ++h) {
    const int j = jb + h * 256 + threadIdx.x;
    valid[h] = j < je;
    jj[h] = valid[h] ? j : jb;
    u0[h] = ldg(N.seg + jj[h]);
    u1[h] = ldg(N.seg + jj[h] + 1);
    if (!valid[h]) u1[h] = u0[h];
  }
  // all K-split partials of w at once (S <= MAXS), summed in split order
  float wpart[kUnitCPT][MAXS];
  {
    const size_t ss = (size_t)N.Bp * N.ncp;
#pragma unroll
    for (int h = 0; h < kUnitCPT; ++h) {
      const float *wp = N.Wws + (size_t)i * N.ncp + jj[h];
#pragma unroll
      for (int t = 0; t < MAXS; ++t) {
        const float v = ldg(wp + (t < N.S ? t : 0) * ss);
        wpart[h][t] = t < N.S ? v : 0.f;
      }
    }
  }
  const double *ci = N.c + (size_t)i * N.n_g, *qi = N.q + (size_t)i * N.n_g;
  double cu[kUnitRounds], qu[kUnitRounds], lo[kUnitRounds], hi[kUnitRounds];
  int uj[kUnitRounds];
#pragma unroll
  for (int a = 0; a < kUnitRounds; ++a) {
    const int u = ub + a * 256 + threadIdx.x;
    const int uc = u < ue ? u : ub;
    cu[a] = ldg(ci + uc);
    qu[a] = ldg(qi + uc);
    lo[a] = ldg(N.pmin + uc);
    hi[a] = ldg(N.pmax + uc);
    uj[a] = ldg(N.ucol + uc);
  }
  const double lam = N.lam[(size_t)par * N.B + i];
  const bool avg = sc->avg_on;
#pragma unroll
  for (int h = 0; h < kUnitCPT; ++h) {
    if (!valid[h]) continue;
    double w = 0.0;
#pragma unroll
    for (int t = 0; t < MAXS; ++t) w += (double)wpart[h][t];
    wcol[jj[h] - jb] = w;
  }
  double x[kUnitCPT], phs = 0.0;
#pragma unroll
  for (int h = 0; h < kUnitCPT; ++h) x[h] = 0.0;
  for (int cs = ub; cs < ue; cs += kUnitChunk) {  // uniform: every block has a unit
    __syncthreads();  // w is in LDS; the previous chunk has been added up
#pragma unroll
    for (int a = 0; a < kUnitRounds; ++a) {
      const int u = cs + a * 256 + threadIdx.x;
      if (u >= ue) continue;
      double cc = cu[a], qq = qu[a], ll = lo[a], hh = hi[a];
      int j = uj[a];
      if (cs != ub) {  // beyond the first chunk (rare): loaded here
        cc = ci[u];
        qq = qi[u];
        ll = N.pmin[u];
        hh = N.pmax[u];
        j = N.ucol[u];
      }
      const double r = cc - lam + wcol[j - jb];
      const double p = inner_min_b(r, qq, ll, hh);
      pch[u - cs] = p;
      phch[u - cs] = r * p + qq * p * p;
      if (avg) N.psum[(size_t)i * N.n_g + u] += p;  // unit u of instance i: one owner
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < kUnitCPT; ++h) {
      const int a0 = max(u0[h], cs), a1 = min(u1[h], cs + kUnitChunk);
      for (int u = a0; u < a1; ++u) {
        x[h] += pch[u - cs];
        phs += phch[u - cs];
      }
    }
  }
  double xs = 0.0;
#pragma unroll
  for (int h = 0; h < kUnitCPT; ++h) {
    if (!valid[h]) continue;
    __bf16 xh, xl;
    split_bf16((float)x[h], &xh, &xl);
    N.X_hi[(size_t)i * N.ldc + jj[h]] = xh;
    N.X_lo[(size_t)i * N.ldc + jj[h]] = xl;
    xs += x[h];
  }
  double sums[2] = {xs, phs};
  block_sums<2>(sums, red);
  if (threadIdx.x == 0) {
    double *up = N.unitpart + (size_t)par * N.ncb * N.Bp * 2 + ((size_t)cb * N.Bp + i) * 2;
    up[0] = sums[0];
    up[1] = sums[1];
    if (blockIdx.x == 0) {
      BIter nx;
      nx.k = sc->it[par].k + 1;
      nx.pending = 1;
      nx.pad = 0;
      sc->it[par ^ 1] = nx;
      if (avg) sc->avg_count += 1;
    }
  }
}

// ---------------------------------------------------------------------------
// F product with the line update in its epilogue.
// ---------------------------------------------------------------------------
// rows of an accumulator whose state is loaded before any of it is stored
constexpr int kEpiChunk = 8;
// row stride (doubles) of the line-term buffer: 33 keeps the half-wavefront
// row writes and the quarter-row reads on few shared banks
constexpr int kTermStride = 33;
static_assert(4 * 16 * kTermStride * 8 <= (int)sizeof(TileLds<32, 128>), "LDS");


template <int BM, int BN, int WM, int WN, bool LOLO>
__device__ __forceinline__ void fgemm_body(const BNet &N, int4 t, const BScal *sc, int par,
                                           const BParams &prm, unsigned char *lds) {
  constexpr int TM = BM / (WM * 32), TN = BN / (WN * 32);
  TileLds<BM, BN> &sm = *reinterpret_cast<TileLds<BM, BN> *>(lds);
  const int m0 = t.y * BM, n0 = t.z * BN;
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  tile_mma<BM, BN, WM, WN, LOLO>(N.X_hi + (size_t)m0 * N.ldc, N.X_lo + (size_t)m0 * N.ldc,
                                 N.ldc, N.P_hi + (size_t)n0 * N.ldc,
                                 N.P_lo + (size_t)n0 * N.ldc, N.ldc, 0, N.ldc, sm, acc,
                                 N.nt_panel != 0);
  const long long k = sc->it[par].k;
  const double kk = (double)k;
  const float a = (float)((prm.decay == 0.0 ? N.alpha : N.alpha / (1.0 + prm.decay * kk)));
  const float rho = (float)N.rho;
  // Adam's bias corrections (pow is costly; the other rules skip it)
  float c1 = 1.f, c2 = 1.f;
  if (prm.rule == DCOPF_RULE_ADAM) {
    c1 = (float)(1.0 - pow(prm.beta1, kk + 1.0));
    c2 = (float)(1.0 - pow(prm.beta2, kk + 1.0));
  }
  const float b1 = (float)prm.beta1, b2 = (float)prm.beta2, eps = (float)prm.eps;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;
  // restrict-qualified views: the loads of a 16-row chunk are issued before
  // any of its stores
  const float *__restrict__ fdp = N.fd32;
  float *__restrict__ mup = N.mu_p;
  float *__restrict__ mum = N.mu_m;
  float *__restrict__ vpp = N.v_p;
  float *__restrict__ vmp = N.v_m;
  float *__restrict__ spp = N.s_p;
  float *__restrict__ smp = N.s_m;
  __bf16 *__restrict__ vhi = N.V_hi;
  __bf16 *__restrict__ vlo = N.V_lo;
  const bool need_v = prm.rule != DCOPF_RULE_ADAGRAD, need_s = prm.rule != DCOPF_RULE_GDM;
  // the line terms of a chunk's 16 instance rows (8 per half-wavefront) go
  // through this wavefront's [16][33] FP64 buffer in the tile's LDS, free
  // once every wavefront has left the K loop
  __syncthreads();
  double *tb = reinterpret_cast<double *>(lds) + wave * 16 * kTermStride;
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int nsub = n0 + (wn * TN + j) * 32;  // first line of this 32-line tile
    const int line = nsub + (lane & 31);
    const bool lvalid = line < N.n_l;
    const float fl = lvalid ? N.flim32[line] : 0.f;
#pragma unroll
    for (int ii = 0; ii < TM; ++ii) {
      const int mb = m0 + (wm * TM + ii) * 32;
#pragma unroll
      for (int h = 0; h < 16; h += kEpiChunk) {
      float fd[kEpiChunk], mp[kEpiChunk], mm[kEpiChunk], v1[kEpiChunk], v2[kEpiChunk],
          s1[kEpiChunk], s2[kEpiChunk];
#pragma unroll
      for (int c = 0; c < kEpiChunk; ++c) {
        // clamped (in-range) offsets: every load goes out before any wait;
        // rows outside the batch or lines past n_l are never stored
        const int e = h + c;
        const int i = mb + mfma32_row(e, lane);
        const unsigned bo = ((unsigned)(i < N.B ? i : 0) * (unsigned)N.ldl +
                             (unsigned)(lvalid ? line : 0)) * 4u;
        fd[c] = ld_at(fdp, bo);
        mp[c] = ld_at(mup, bo);
        mm[c] = ld_at(mum, bo);
        v1[c] = v2[c] = s1[c] = s2[c] = 0.f;
      }
      if (need_v)
#pragma unroll
        for (int c = 0; c < kEpiChunk; ++c) {
          const int i = mb + mfma32_row(h + c, lane);
          const unsigned bo = ((unsigned)(i < N.B ? i : 0) * (unsigned)N.ldl +
                               (unsigned)(lvalid ? line : 0)) * 4u;
          v1[c] = ld_at(vpp, bo);
          v2[c] = ld_at(vmp, bo);
        }
      if (need_s)
#pragma unroll
        for (int c = 0; c < kEpiChunk; ++c) {
          const int i = mb + mfma32_row(h + c, lane);
          const unsigned bo = ((unsigned)(i < N.B ? i : 0) * (unsigned)N.ldl +
                               (unsigned)(lvalid ? line : 0)) * 4u;
          s1[c] = ld_at(spp, bo);
          s2[c] = ld_at(smp, bo);
        }
#pragma unroll
      for (int c = 0; c < kEpiChunk; ++c) {
        const int e = h + c;
        const int i = mb + mfma32_row(e, lane);
        const bool ok = lvalid && i < N.B;
        const unsigned bo = ((unsigned)i * (unsigned)N.ldl + (unsigned)line) * 4u;
        const float F = acc[ii][j][e] - fd[c];
        const float gp = F - fl, gm = -F - fl;
        double term = (double)(mp[c] - mm[c]) * (double)fd[c] + (double)(mp[c] + mm[c]) * (double)fl;
        float np_, nm_;
        if (prm.rule == DCOPF_RULE_GDM) {
          const float vp = rho * v1[c] + a * gp, vm = rho * v2[c] + a * gm;
          if (ok) {
            st_at(vpp, bo, vp);
            st_at(vmp, bo, vm);
          }
          np_ = mp[c] + vp;
          nm_ = mm[c] + vm;
          if (prm.literal) {
            np_ += a * gp;
            nm_ += a * gm;
          }
        } else if (prm.rule == DCOPF_RULE_ADAM) {
          const float m1 = b1 * v1[c] + (1.f - b1) * gp;
          const float m2 = b1 * v2[c] + (1.f - b1) * gm;
          const float q1 = b2 * s1[c] + (1.f - b2) * gp * gp;
          const float q2 = b2 * s2[c] + (1.f - b2) * gm * gm;
          if (ok) {
            st_at(vpp, bo, m1);
            st_at(vmp, bo, m2);
            st_at(spp, bo, q1);
            st_at(smp, bo, q2);
          }
          np_ = mp[c] + a * (m1 / c1) / (sqrtf(q1 / c2) + eps);
          nm_ = mm[c] + a * (m2 / c1) / (sqrtf(q2 / c2) + eps);
        } else {
          const float q1 = s1[c] + gp * gp, q2 = s2[c] + gm * gm;
          if (ok) {
            st_at(spp, bo, q1);
            st_at(smp, bo, q2);
          }
          np_ = mp[c] + a * gp / (sqrtf(q1) + eps);
          nm_ = mm[c] + a * gm / (sqrtf(q2) + eps);
        }
        np_ = fmaxf(np_, 0.f);
        nm_ = fmaxf(nm_, 0.f);
        if (ok) {
          st_at(mup, bo, np_);
          st_at(mum, bo, nm_);
          __bf16 hi, lo;
          split_bf16(np_ - nm_, &hi, &lo);
          st_at(vhi, bo >> 1, hi);
          st_at(vlo, bo >> 1, lo);
        }
        if (!ok) term = 0.0;
        tb[(c + 8 * (lane >> 5)) * kTermStride + (lane & 31)] = term;
      }
      // line terms of each instance row summed over the 32 lines of this
      // tile: lane (row r, quarter q) adds lines 8q .. 8q + 7 in order, then
      // the four quarters are added (in the same order on every lane)
      {
        const int r = lane & 15, q = lane >> 4;
        double sum = 0.0;
#pragma unroll
        for (int x = 0; x < 8; ++x) sum += tb[r * kTermStride + q * 8 + x];
        sum += __shfl_xor(sum, 16, kWave);
        sum += __shfl_xor(sum, 32, kWave);
        const int i = mb + mfma32_row(h + (r & 7), (r >> 3) * 32);
        if (q == 0 && i < N.B) N.linepart[(size_t)(nsub / 32) * N.Bp + i] = sum;
      }
      }
    }
  }
}

template <bool LOLO>
__global__ __launch_bounds__(256) void fgemm_kernel(const BNet *__restrict__ nets,
                                                    const int4 *__restrict__ tiles,
                                                    const BScal *sc, int par, BParams prm) {
  __shared__ __align__(16) unsigned char lds[kTileLdsBytes];
  const int4 t = tiles[blockIdx.x];
  const BNet &N = nets[t.x];
#define DCOPF_FBODY(BM, BN, WM, WN) fgemm_body<BM, BN, WM, WN, LOLO>(N, t, sc, par, prm, lds)
  DCOPF_TILE_SWITCH(N.cfg_f, DCOPF_FBODY)
#undef DCOPF_FBODY
}

// End of a step call: fold the last iteration (k_prev, parity pp) of every
// instance into the lambda slot of the next iteration (parity pp ^ 1), which
// is then no longer pending.
__global__ __launch_bounds__(256) void bfinal_kernel(const BNet *__restrict__ nets,
                                                     const int2 *__restrict__ inst_tab,
                                                     BScal *sc, int pp, long long k_prev,
                                                     BParams prm, double *__restrict__ gam_ring,
                                                     long long gmask, int n_total) {
  const int slot = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (slot < n_total) {
    const int2 e = inst_tab[slot];
    fold_wave(nets[e.x], e.y, pp, k_prev, prm, gam_ring, gmask, n_total);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->it[pp ^ 1].pending = 0;
}

// ---------------------------------------------------------------------------
// FP64 products (exact bound, and f_d = H d at setup):
// C[m][n] = sum_k A[m][k] B[n][k], A [Mp][ld], B [Np][ld], C [Mp][ldo];
// Mp multiple of 64, Np multiple of 16, ld multiple of 4.  Four wavefronts
// per workgroup along M, 16 x 16 tiles, v_mfma_f64_16x16x4f64.
// ---------------------------------------------------------------------------
constexpr int kDgemmAhead = 16;

__global__ __launch_bounds__(256) void dgemm_nt_kernel(const double *__restrict__ A,
                                                       const double *__restrict__ Bm,
                                                       double *__restrict__ C, int ld,
                                                       int ldo, int Mp) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = (blockIdx.y * 4 + wave) * 16, n0 = blockIdx.x * 16;
  if (m0 >= Mp) return;
  const int r = lane & 15, kk = lane >> 4;
  const double *a = A + (size_t)(m0 + r) * ld + kk;
  const double *b = Bm + (size_t)(n0 + r) * ld + kk;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  // kDgemmAhead K steps of operands are loaded before their products, so a
  // wavefront waits once per kDgemmAhead steps instead of once per step; the
  // products are accumulated in the same K order either way
  int k = 0;
  for (; k + 4 * kDgemmAhead <= ld; k += 4 * kDgemmAhead) {
    double av[kDgemmAhead], bv[kDgemmAhead];
#pragma unroll
    for (int u = 0; u < kDgemmAhead; ++u) {
      av[u] = a[k + 4 * u];
      bv[u] = b[k + 4 * u];
    }
#pragma unroll
    for (int u = 0; u < kDgemmAhead; ++u)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
  }
  for (; k < ld; k += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k], b[k], acc, 0, 0, 0);
  // register j of lane l holds row 4 j + l / 16, column l % 16
#pragma unroll
  for (int j = 0; j < 4; ++j) C[(size_t)(m0 + 4 * j + kk) * ldo + n0 + r] = acc[j];
}

// V64[i][l] = mu+ - mu- (FP64 from the FP32 state) for the exact bound.
__global__ void make_v64_kernel(const float *mu_p, const float *mu_m, int B, int n_l, int ldl,
                                double *V64) {
  const int i = blockIdx.y;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n_l; l += gridDim.x * blockDim.x)
    V64[(size_t)i * ldl + l] =
        (double)mu_p[(size_t)i * ldl + l] - (double)mu_m[(size_t)i * ldl + l];
}

// Exact bound of instance i (one workgroup): sum over units of phi with the
// FP64 w, plus lambda D, minus the FP64 line terms.
__global__ __launch_bounds__(256) void bound_inst_kernel(BNet N, int par) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const double lam = N.lam[(size_t)par * N.B + i];
  const double *ci = N.c + (size_t)i * N.n_g, *qi = N.q + (size_t)i * N.n_g;
  double phis = 0.0, lines = 0.0;
  for (int j = threadIdx.x; j < N.n_c; j += blockDim.x) {
    const double w = N.W64[(size_t)i * N.ncp + j];
    for (int u = N.seg[j]; u < N.seg[j + 1]; ++u) {
      const double r = ci[u] - lam + w;
      const double p = inner_min_b(r, qi[u], N.pmin[u], N.pmax[u]);
      phis += r * p + qi[u] * p * p;
    }
  }
  for (int l = threadIdx.x; l < N.n_l; l += blockDim.x) {
    const double mp = N.mu_p[(size_t)i * N.ldl + l], mm = N.mu_m[(size_t)i * N.ldl + l];
    lines += (mp - mm) * N.fd64[(size_t)i * N.n_l + l] + (mp + mm) * N.flim64[l];
  }
  phis = block_sum(phis, red);
  lines = block_sum(lines, red);
  if (threadIdx.x == 0) N.bound[i] = phis + lam * N.D[i] - lines;
}

// ---- primal average (an extension) ------------------------------------------
constexpr int kPrimalColBlocks = 16;  // column blocks per instance in the evaluation

// Workgroup (column block, instance): pbar per unit, the averaged injection
// xbar per column (FP64, zero in the padding), and the block's cost and
// generation.
__global__ __launch_bounds__(256) void bprimal_cols_kernel(BNet N, const BScal *sc,
                                                           double *__restrict__ part) {
  __shared__ double red[2 * 4];
  const int i = blockIdx.y;
  const double n = (double)sc->avg_count;
  const double *ci = N.c + (size_t)i * N.n_g, *qi = N.q + (size_t)i * N.n_g;
  double v[2] = {0.0, 0.0};
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N.ldc; j += gridDim.x * blockDim.x) {
    double xs = 0.0;
    if (j < N.n_c)
      for (int u = N.seg[j]; u < N.seg[j + 1]; ++u) {
        const double p = N.psum[(size_t)i * N.n_g + u] / n;
        N.pbar[(size_t)i * N.n_g + u] = p;
        v[0] += ci[u] * p + qi[u] * p * p;
        xs += p;
      }
    N.X64[(size_t)i * N.ldc + j] = xs;
    v[1] += xs;
  }
  block_sums<2>(v, red);
  if (threadIdx.x == 0) {
    part[((size_t)i * gridDim.x + blockIdx.x) * 2] = v[0];
    part[((size_t)i * gridDim.x + blockIdx.x) * 2 + 1] = v[1];
  }
}

// One workgroup per instance: F = (P xbar) - f_d against the limits (FP64),
// then the instance's cost, balance and overloads in a fixed order.
__global__ __launch_bounds__(256) void bprimal_inst_kernel(BNet N, const BScal *sc,
                                                           const double *__restrict__ part,
                                                           int gc, double *__restrict__ out) {
  __shared__ double red[2 * 4];
  __shared__ double mx_s[4];
  const int i = blockIdx.x;
  double mx = 0.0, v[2] = {0.0, 0.0};  // sum of overloads, their count
  for (int l = threadIdx.x; l < N.n_l; l += blockDim.x) {
    const double F = N.F64[(size_t)i * N.nlp + l] - N.fd64[(size_t)i * N.n_l + l];
    const double o1 = fmax(F - N.flim64[l], 0.0), o2 = fmax(-F - N.flim64[l], 0.0);
    mx = fmax(mx, fmax(o1, o2));
    v[0] += o1 + o2;
    v[1] += (o1 > 0.0 ? 1.0 : 0.0) + (o2 > 0.0 ? 1.0 : 0.0);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
  if (threadIdx.x % kWave == 0) mx_s[threadIdx.x / kWave] = mx;
  block_sums<2>(v, red);  // its barriers also publish mx_s
  if (threadIdx.x == 0) {
    double cost = 0.0, gen = 0.0, m = 0.0;
    for (int b = 0; b < gc; ++b) {
      cost += part[((size_t)i * gc + b) * 2];
      gen += part[((size_t)i * gc + b) * 2 + 1];
    }
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) m = fmax(m, mx_s[w]);
    double *o = out + (size_t)i * 5;
    o[0] = cost;
    o[1] = N.D[i] - gen;
    o[2] = m;
    o[3] = v[0];
    o[4] = v[1];
  }
}

// ---------------------------------------------------------------------------
// Repair of every instance's primal candidate into a feasible dispatch (not
// in the paper): the rounds of the single-instance repair for all instances
// of a network at once, grid rows being instances.  Per round: x and the
// weights per column (FP64), F = X P64^T for every instance (FP64 matrix
// cores), one workgroup per instance for the ordered append to its active
// set and the targets, then the Gram matrices (one wavefront per entry),
// one workgroup per instance for the Cholesky solve, and the step.  An
// instance whose rounds have ended (stop) is left untouched.
// ---------------------------------------------------------------------------
constexpr int kBRepRows = 256;         // active lines + the balance row
constexpr double kBRepMargin = 1e-6;   // MW inside each held limit
constexpr double kBRepBalTol = 1e-9;   // of max(1, 1^T d)
constexpr double kBRepFloor = 1e-3;    // weight floor, of a unit's range
constexpr double kBRepRidge = 1e-12;   // of the largest Gram diagonal

struct BRepState {
  double beta;       // 1^T d - 1^T p of the evaluated iterate
  int n_viol;        // violated line directions
  int m_old, m;      // active lines before / after this evaluation
  int overflow;      // more than kBRepRows - 1 lines would be active
  int done;          // stop rule met
  int fail;          // a Gram matrix was not positive definite
  int rounds;        // correction steps taken
  int stop;          // no further step for this instance
};

__device__ __forceinline__ double brep_weight(double p, double lo, double hi) {
  return fmax(fmin(p - lo, hi - p), kBRepFloor * (hi - lo));
}

// p = p0c = clip(src); no line active; zero state.
__global__ void brep_init_kernel(BNet N, const double *__restrict__ src, double *__restrict__ p,
                                 double *__restrict__ p0c, int *__restrict__ pos,
                                 BRepState *st) {
  const int i = blockIdx.y;
  const int n = max(N.n_g, N.n_l);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    if (e < N.n_g) {
      const size_t k = (size_t)i * N.n_g + e;
      const double v = fmin(fmax(src[k], N.pmin[e]), N.pmax[e]);
      p[k] = v;
      p0c[k] = v;
    }
    if (e < N.n_l) pos[(size_t)i * N.n_l + e] = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    BRepState s{};
    st[i] = s;
  }
}

// Per instance and column: x (into X64, zero beyond n_c), the column's
// weight W, block partials of the cost and the generation.
__global__ __launch_bounds__(256) void brep_cols_kernel(BNet N, const double *__restrict__ p,
                                                        double *__restrict__ W,
                                                        double *__restrict__ part) {
  __shared__ double red[2 * 4];
  const int i = blockIdx.y;
  const double *pi = p + (size_t)i * N.n_g;
  const double *ci = N.c + (size_t)i * N.n_g, *qi = N.q + (size_t)i * N.n_g;
  double v[2] = {0.0, 0.0};
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N.ldc; j += gridDim.x * blockDim.x) {
    double xs = 0.0, ws = 0.0;
    if (j < N.n_c)
      for (int u = N.seg[j]; u < N.seg[j + 1]; ++u) {
        const double pu = pi[u];
        v[0] += ci[u] * pu + qi[u] * pu * pu;
        xs += pu;
        ws += brep_weight(pu, N.pmin[u], N.pmax[u]);
      }
    N.X64[(size_t)i * N.ldc + j] = xs;
    W[(size_t)i * N.ldc + j] = ws;
    v[1] += xs;
  }
  block_sums<2>(v, red);
  if (threadIdx.x == 0) {
    part[((size_t)i * gridDim.x + blockIdx.x) * 2] = v[0];
    part[((size_t)i * gridDim.x + blockIdx.x) * 2 + 1] = v[1];
  }
}

// One workgroup of 256 per instance: violations of F = F64 - f_d, ordered
// append (rows, sgn; pos[l] = row of line l or -1), targets t[0..m]
// (t[m]: balance), the stop decision.
__global__ __launch_bounds__(256) void brep_active_kernel(
    BNet N, const double *__restrict__ part, int gc, int max_rounds, int *__restrict__ pos,
    int *__restrict__ rows, int *__restrict__ sgn, double *__restrict__ t, BRepState *st) {
  __shared__ int wave_new[4];
  __shared__ int m_s, viol_s;
  __shared__ double beta_s;
  __shared__ BRepState s0;
  const int i = blockIdx.x, tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  if (tid == 0) s0 = st[i];
  __syncthreads();
  if (s0.stop) return;
  if (tid == 0) {
    double gen = 0.0;
    for (int b = 0; b < gc; ++b) gen += part[((size_t)i * gc + b) * 2 + 1];
    beta_s = N.D[i] - gen;
    m_s = s0.m;
    viol_s = 0;
  }
  __syncthreads();
  int *posi = pos + (size_t)i * N.n_l;
  int *rowsi = rows + (size_t)i * kBRepRows, *sgni = sgn + (size_t)i * kBRepRows;
  const double *Fi = N.F64 + (size_t)i * N.nlp, *fdi = N.fd64 + (size_t)i * N.n_l;
  const int m_old = m_s;
  for (int base = 0; base < N.n_l; base += 256) {
    const int l = base + tid;
    int sigma = 0;
    if (l < N.n_l) {
      const double Fl = Fi[l] - fdi[l];
      if (Fl - N.flim64[l] > 0.0)
        sigma = 1;
      else if (-Fl - N.flim64[l] > 0.0)
        sigma = -1;
    }
    bool fresh = false;
    if (sigma != 0) {
      const int r = posi[l];
      if (r >= 0)
        sgni[r] = sigma;  // held line: keep its row, take this direction
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
      if (r < kBRepRows - 1) {
        rowsi[r] = l;
        sgni[r] = sigma;
        posi[l] = r;
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
  const bool over = m > kBRepRows - 1;
  if (over) m = kBRepRows - 1;
  double *ti = t + (size_t)i * kBRepRows;
  for (int r = tid; r < m; r += blockDim.x) {
    const int l = rowsi[r];
    const double Fl = Fi[l] - fdi[l];
    ti[r] = sgni[r] > 0 ? (-kBRepMargin - (Fl - N.flim64[l])) : (kBRepMargin + (-Fl - N.flim64[l]));
  }
  if (tid == 0) {
    ti[m] = beta_s;
    BRepState s = s0;
    s.beta = beta_s;
    s.n_viol = viol_s;
    s.m_old = m_old;
    s.m = m;
    s.overflow = (over || s0.overflow) ? 1 : 0;
    s.done = (viol_s == 0 && fabs(beta_s) <= kBRepBalTol * fmax(1.0, fabs(N.D[i]))) ? 1 : 0;
    s.stop = (s.done || s.fail || s.overflow || s.rounds >= max_rounds) ? 1 : 0;
    st[i] = s;
  }
}

// A[i][r][c] = P[rows[i][r]][c] for the rows that joined (x blocks: column
// chunk by new row).
__global__ void brep_gather_kernel(BNet N, const int *__restrict__ rows, const BRepState *st,
                                   int ccb, double *__restrict__ A) {
  const int i = blockIdx.y;
  const BRepState s = st[i];
  const int r = s.m_old + (int)blockIdx.x / ccb;
  if (s.stop || r >= s.m) return;
  const int l = rows[(size_t)i * kBRepRows + r];
  const int c = ((int)blockIdx.x % ccb) * blockDim.x + threadIdx.x;
  if (c < N.ldc)
    A[((size_t)i * kBRepRows + r) * N.ldc + c] = N.P64[(size_t)l * N.ldc + c];
}

// G[i][a][b] (a >= b < m_i + 1; row m_i is the balance row of ones): one
// wavefront per entry.
__global__ __launch_bounds__(256) void brep_gram_kernel(BNet N, const double *__restrict__ A,
                                                        const double *__restrict__ W,
                                                        const BRepState *st,
                                                        double *__restrict__ G) {
  const int i = blockIdx.y;
  const BRepState s = st[i];
  if (s.stop) return;
  const int m = s.m, n = m + 1;
  const long long k = (long long)blockIdx.x * 4 + threadIdx.x / kWave;
  if (k >= (long long)n * (n + 1) / 2) return;
  int a = (int)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
  while ((long long)(a + 1) * (a + 2) / 2 <= k) ++a;
  while ((long long)a * (a + 1) / 2 > k) --a;
  const int b = (int)(k - (long long)a * (a + 1) / 2);
  const int lane = threadIdx.x % kWave;
  const double *Ai = A + (size_t)i * kBRepRows * N.ldc;
  const double *aa = Ai + (size_t)a * N.ldc, *ab = Ai + (size_t)b * N.ldc;
  const double *Wi = W + (size_t)i * N.ldc;
  double sum = 0.0;
  for (int c = lane; c < N.n_c; c += kWave) {
    const double x = a < m ? aa[c] : 1.0, y = b < m ? ab[c] : 1.0;
    sum += Wi[c] * x * y;
  }
  sum = wave_sum(sum);
  if (lane == 0) G[((size_t)i * kBRepRows + a) * kBRepRows + b] = sum;
}

// One workgroup per instance: the working-set solve of its step (ws_solve).
__global__ __launch_bounds__(1024) void brep_solve_kernel(const double *__restrict__ G,
                                                          const double *__restrict__ t,
                                                          const int *__restrict__ sgn,
                                                          double *__restrict__ L,
                                                          double *__restrict__ y,
                                                          BRepState *st) {
  __shared__ WsShared sh;
  const int i = blockIdx.x;
  if (st[i].stop) return;
  const size_t g0 = (size_t)i * kBRepRows * kBRepRows, r0 = (size_t)i * kBRepRows;
  const bool ok = ws_solve<kBRepRows>(G + g0, t + r0, sgn + r0, st[i].m, L + g0, y + r0,
                                      kBRepMargin, kBRepRidge, sh);
  if (!ok && threadIdx.x == 0) st[i].fail = 1;
}

// p_u += w_u z_c (z_c = sum_r y_r A[r][c] + y_m), clipped to the box; one
// more round for the instance.
__global__ __launch_bounds__(256) void brep_step_kernel(BNet N, const double *__restrict__ A,
                                                        const double *__restrict__ y,
                                                        BRepState *st, double *__restrict__ p) {
  const int i = blockIdx.y;
  const BRepState s = st[i];
  if (s.stop || s.fail) return;
  const int m = s.m;
  const double *Ai = A + (size_t)i * kBRepRows * N.ldc;
  const double *yi = y + (size_t)i * kBRepRows;
  double *pi = p + (size_t)i * N.n_g;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N.n_c; j += gridDim.x * blockDim.x) {
    double z = 0.0;
    for (int r = 0; r < m; ++r) z += yi[r] * Ai[(size_t)r * N.ldc + j];
    z += yi[m];
    for (int u = N.seg[j]; u < N.seg[j + 1]; ++u) {
      const double pu = pi[u];
      pi[u] = fmin(fmax(pu + brep_weight(pu, N.pmin[u], N.pmax[u]) * z, N.pmin[u]), N.pmax[u]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st[i].rounds = s.rounds + 1;
}

// One workgroup per instance: cost, balance, largest overload and largest
// shift of the final iterate; out[i][0..3].
__global__ __launch_bounds__(256) void brep_final_kernel(BNet N, const double *__restrict__ part,
                                                         int gc, const double *__restrict__ p,
                                                         const double *__restrict__ p0c,
                                                         double *__restrict__ out) {
  __shared__ double mo_s[4], sh_s[4];
  const int i = blockIdx.x;
  const double *Fi = N.F64 + (size_t)i * N.nlp, *fdi = N.fd64 + (size_t)i * N.n_l;
  double mo = 0.0, sh = 0.0;
  for (int l = threadIdx.x; l < N.n_l; l += blockDim.x) {
    const double F = Fi[l] - fdi[l];
    mo = fmax(mo, fmax(F - N.flim64[l], -F - N.flim64[l]));
  }
  for (int u = threadIdx.x; u < N.n_g; u += blockDim.x)
    sh = fmax(sh, fabs(p[(size_t)i * N.n_g + u] - p0c[(size_t)i * N.n_g + u]));
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    mo = fmax(mo, __shfl_xor(mo, off, kWave));
    sh = fmax(sh, __shfl_xor(sh, off, kWave));
  }
  if (threadIdx.x % kWave == 0) {
    mo_s[threadIdx.x / kWave] = mo;
    sh_s[threadIdx.x / kWave] = sh;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double cost = 0.0, gen = 0.0;
  for (int b = 0; b < gc; ++b) {
    cost += part[((size_t)i * gc + b) * 2];
    gen += part[((size_t)i * gc + b) * 2 + 1];
  }
  mo = 0.0;
  sh = 0.0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
    mo = fmax(mo, mo_s[w]);
    sh = fmax(sh, sh_s[w]);
  }
  out[(size_t)i * 4] = cost;
  out[(size_t)i * 4 + 1] = N.D[i] - gen;
  out[(size_t)i * 4 + 2] = mo;
  out[(size_t)i * 4 + 3] = sh;
}

// Start multipliers of every instance from rows of a device array (the warm
// start network's output): mu+ = max(0, Y[i][l]), mu- = max(0, Y[i][n_l + l])
// into the FP32 state (zero padding), lambda = Y[i][2 n_l] into slot 0;
// bad = 1 on a value that is not finite.
__global__ void bset_start_kernel(BNet N, const float *__restrict__ Y, int ld, int *bad) {
  const int i = blockIdx.y;
  const float *yi = Y + (size_t)i * ld;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < N.ldl; l += gridDim.x * blockDim.x) {
    float a = 0.f, c = 0.f;
    if (l < N.n_l) {
      a = yi[l];
      c = yi[N.n_l + l];
      if (!isfinite(a) || !isfinite(c)) *bad = 1;
      a = fmaxf(a, 0.f);
      c = fmaxf(c, 0.f);
    }
    N.mu_p[(size_t)i * N.ldl + l] = a;
    N.mu_m[(size_t)i * N.ldl + l] = c;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const float lam = yi[2 * N.n_l];
    if (!isfinite(lam)) *bad = 1;
    N.lam[i] = (double)lam;
  }
}

// Instance i of `dst` takes the whole state of instance i of `src` when the
// exact bound of `src`'s is larger (both evaluated at the same iteration):
// multipliers, optimiser state, the split of v, the bound and the primal
// sums; kept[i] says which.  Grid: (column blocks, instances).
__global__ void badopt_kernel(BNet dst, BNet src, int slot, int *__restrict__ kept) {
  const int i = blockIdx.y;
  const bool take = src.bound[i] > dst.bound[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) kept[i] = take ? 1 : 0;
  if (!take) return;
  const size_t row = (size_t)i * dst.ldl;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < dst.ldl; l += gridDim.x * blockDim.x) {
    dst.mu_p[row + l] = src.mu_p[row + l];
    dst.mu_m[row + l] = src.mu_m[row + l];
    dst.v_p[row + l] = src.v_p[row + l];
    dst.v_m[row + l] = src.v_m[row + l];
    dst.s_p[row + l] = src.s_p[row + l];
    dst.s_m[row + l] = src.s_m[row + l];
    dst.V_hi[row + l] = src.V_hi[row + l];
    dst.V_lo[row + l] = src.V_lo[row + l];
  }
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < dst.n_g; g += gridDim.x * blockDim.x)
    dst.psum[(size_t)i * dst.n_g + g] = src.psum[(size_t)i * dst.n_g + g];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const size_t a = (size_t)slot * dst.B + i;
    dst.lam[a] = src.lam[a];
    dst.vlam[a] = src.vlam[a];
    dst.slam[a] = src.slam[a];
    dst.bound[i] = src.bound[i];
  }
}

// ---- setup -----------------------------------------------------------------
// tmp[l][j] = H[l][cols[j]] (zero padded to [nlp][ldc]) in FP64.
__global__ void bgather_kernel(const double *__restrict__ H, int n_bus, int n_l,
                               const int *__restrict__ cols, int n_c, int ldc,
                               double *__restrict__ out) {
  const int l = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ldc; j += gridDim.x * blockDim.x)
    out[(size_t)l * ldc + j] = (l < n_l && j < n_c) ? H[(size_t)l * n_bus + cols[j]] : 0.0;
}

// outT[j][l] = in[l][j] for j < rowsT, l < ldT (zero beyond the input).
__global__ void btranspose_kernel(const double *__restrict__ in, int rows_in, int ld_in,
                                  int rowsT, int ldT, double *__restrict__ outT) {
  __shared__ double tile[32][33];
  const int j0 = blockIdx.x * 32, l0 = blockIdx.y * 32;
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int l = l0 + r, j = j0 + threadIdx.x;
    tile[r][threadIdx.x] = (l < rows_in && j < ld_in) ? in[(size_t)l * ld_in + j] : 0.0;
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int j = j0 + r, l = l0 + threadIdx.x;
    if (j < rowsT && l < ldT) outT[(size_t)j * ldT + l] = tile[threadIdx.x][r];
  }
}

__global__ void bsplit_kernel(const double *__restrict__ in, size_t n, __bf16 *__restrict__ hi,
                              __bf16 *__restrict__ lo) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    const double v = in[t];
    const __bf16 h = (__bf16)v;
    hi[t] = h;
    lo[t] = (__bf16)(v - (double)(float)h);
  }
}

// f_d from the FP64 product tmp [Bp][nlp16]: fd64 [B][n_l], fd32 [B][ldl]
__global__ void bfd_kernel(const double *__restrict__ tmp, int ldt, int B, int n_l, int ldl,
                           double *__restrict__ fd64, float *__restrict__ fd32) {
  const int i = blockIdx.y;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n_l; l += gridDim.x * blockDim.x) {
    const double v = tmp[(size_t)i * ldt + l];
    fd64[(size_t)i * n_l + l] = v;
    fd32[(size_t)i * ldl + l] = (float)v;
  }
}

// V hi/lo from the FP32 state (after a warm start).
__global__ void bmake_v_kernel(const float *mu_p, const float *mu_m, int B, int n_l, int ldl,
                               __bf16 *V_hi, __bf16 *V_lo) {
  const int i = blockIdx.y;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n_l; l += gridDim.x * blockDim.x) {
    const size_t idx = (size_t)i * ldl + l;
    split_bf16(mu_p[idx] - mu_m[idx], V_hi + idx, V_lo + idx);
  }
}

}  // namespace
}  // namespace dcopf

// ===========================================================================
// Host side
// ===========================================================================
using namespace dcopf;

namespace {

struct HostNet {
  BNet d{};  // device pointers (owned) and shapes
  std::vector<int> gperm;  // unit t of the column order is generator gperm[t]
  std::vector<int> seg;    // units of column j: seg[j] .. seg[j+1]-1
  int n_bus = 0;
  // primal repair buffers (allocated by the network's first repair)
  struct Repair {
    double *pin = nullptr, *p = nullptr, *p0c = nullptr, *W = nullptr, *t = nullptr,
           *y = nullptr, *G = nullptr, *L = nullptr, *A = nullptr, *part = nullptr,
           *out = nullptr;
    int *pos = nullptr, *rows = nullptr, *sgn = nullptr;
    BRepState *st = nullptr;
    bool ready = false;
  } rep;
  double best_dummy = 0;
};

template <typename T> T *balloc(DevPool &pool, size_t n, bool *ok) {
  T *p = pool.get_n<T>(n == 0 ? 1 : n);
  if (!p) *ok = false;
  return p;
}

bool finite_all_b(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

struct dcopf_batch_s {
  DevPool pool;  // every device buffer of the batch (the caller's allocator)
  std::vector<HostNet> nets;
  dcopf_batch_opts opts{};
  BParams prm{};
  hipStream_t stream = nullptr;
  BNet *d_nets = nullptr;
  int4 *d_wtiles = nullptr, *d_ftiles = nullptr;
  int2 *d_inst = nullptr;   // (network, instance) per instance
  int4 *d_units = nullptr;  // per unit-pass workgroup: (network | column block << 16,
                            // instance, first unit, end of its units)
  int n_wtiles = 0, n_ftiles = 0, n_total = 0, n_units = 0;
  BScal *sc = nullptr;
  double *gam = nullptr;
  long long gcap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_iters = 0;
  long long iters = 0;
  std::vector<double> best;
  std::vector<long long> best_iter;
};

namespace {

void free_batch(dcopf_batch_s *b) {
  if (!b) return;
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->pool.release_all();
  delete b;
}

// Workgroup i of a launch runs on XCD i % 8 (round-robin dispatch).  The M
// tiles that read the same panel block get ids that differ by a multiple of
// 8 and are adjacent in dispatch order, so one XCD reads the block from HBM
// and its other M tiles hit that XCD's L2.
constexpr int kXcds = 8;

void push_xcd_grouped(std::vector<int4> *out, int k, int Mt,
                      const std::vector<std::pair<int, int>> &pblocks) {
  const int G = (int)pblocks.size();
  for (int g0 = 0; g0 < G; g0 += kXcds) {
    const int r = std::min(kXcds, G - g0);
    for (int m = 0; m < Mt; ++m)
      for (int x = 0; x < r; ++x)
        out->push_back(make_int4(k, m, pblocks[g0 + x].first, pblocks[g0 + x].second));
  }
}

// tile tables from the per-network shapes; the networks with the longest
// K loops first
void build_tables(const std::vector<HostNet> &nets, const std::vector<int> &which,
                  std::vector<int4> *wt, std::vector<int4> *ft) {
  wt->clear();
  ft->clear();
  std::vector<int> order = which;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return nets[a].d.kchunk > nets[b].d.kchunk;
  });
  // tile (m, n, s) covers rows m BM .. m BM + BM - 1, columns n BN .. + BN - 1
  // and K split s; the padded extents (multiples of 128) contain every tile
  for (int k : order) {
    const BNet &N = nets[k].d;
    const int BM = kTileBM[N.cfg_w], BN = kTileBN[N.cfg_w];
    const int Mt = (N.B + BM - 1) / BM, Nt = (N.n_c + BN - 1) / BN;
    std::vector<std::pair<int, int>> pb;
    for (int n = 0; n < Nt; ++n)
      for (int s = 0; s < N.S; ++s) pb.emplace_back(n, s);
    push_xcd_grouped(wt, k, Mt, pb);
  }
  std::vector<int> forder = which;
  std::stable_sort(forder.begin(), forder.end(), [&](int a, int b) {
    return nets[a].d.ldc > nets[b].d.ldc;
  });
  for (int k : forder) {
    const BNet &N = nets[k].d;
    const int BM = kTileBM[N.cfg_f], BN = kTileBN[N.cfg_f];
    const int Mt = (N.B + BM - 1) / BM, Nt = (N.n_l + BN - 1) / BN;
    std::vector<std::pair<int, int>> pb;
    for (int n = 0; n < Nt; ++n) pb.emplace_back(n, 0);
    push_xcd_grouped(ft, k, Mt, pb);
  }
}

void set_split(BNet &N, int S) {
  const int kblocks = N.ldl / 64;
  S = std::max(1, std::min(std::min(S, kblocks), kMaxSplit));
  N.kchunk = (kblocks + S - 1) / S * 64;
  N.S = (N.ldl + N.kchunk - 1) / N.kchunk;
}

// the three passes of one iteration; with events e0/e1 the launch records
// the dispatch's own start and end
void launch_w(dcopf_batch_s *b, hipStream_t s, const int4 *tiles, int n, int par,
              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  // the tiles, then one fold workgroup per four instances
  const int nf = (b->n_total + 3) / 4;
  (void)launch_k(b->opts.lolo ? wgemm_kernel<true> : wgemm_kernel<false>, dim3(n + nf), dim3(256),
                 0, s, e0, e1, b->d_nets, tiles, n, b->d_inst, b->sc, par, b->prm, b->gam,
                 b->gcap - 1, b->n_total);
}

void launch_u(dcopf_batch_s *b, hipStream_t s, int par, hipEvent_t e0 = nullptr,
              hipEvent_t e1 = nullptr) {
  int maxs = 1;
  for (auto &n : b->nets) maxs = std::max(maxs, n.d.S);
  auto kern = maxs <= 8 ? units_kernel<8> : (maxs <= 16 ? units_kernel<16> : units_kernel<32>);
  (void)launch_k(kern, dim3(b->n_units), dim3(256), 0, s, e0, e1, b->d_nets, b->d_units,
                 b->sc, par);
}

void launch_f(dcopf_batch_s *b, hipStream_t s, const int4 *tiles, int n, int par,
              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  if (n == 0) return;
  (void)launch_k(b->opts.lolo ? fgemm_kernel<true> : fgemm_kernel<false>, dim3(n), dim3(256), 0,
                 s, e0, e1, b->d_nets, tiles, b->sc, par, b->prm);
}

void launch_iters_b(dcopf_batch_s *b, hipStream_t s, long long first, int64_t n) {
  for (int64_t t = 0; t < n; ++t) {
    const int par = (int)((first + t) & 1);
    launch_w(b, s, b->d_wtiles, b->n_wtiles, par);
    launch_u(b, s, par);
    launch_f(b, s, b->d_ftiles, b->n_ftiles, par);
  }
}

void launch_final_b(dcopf_batch_s *b, hipStream_t s) {
  if (b->iters <= 0) return;
  const int pp = (int)((b->iters - 1) & 1);  // parity of the last iteration
  bfinal_kernel<<<(b->n_total + 3) / 4, 256, 0, s>>>(b->d_nets, b->d_inst, b->sc, pp, b->iters - 1,
                                                     b->prm, b->gam, b->gcap - 1, b->n_total);
}

// cold start (multipliers, optimiser state, V) of network `only`, or of
// every network when only < 0; the batch's iteration counter restarts at k0
hipError_t reset_state(dcopf_batch_s *b, long long k0, int only = -1) {
  hipError_t e = hipSuccess;
  for (size_t k = 0; k < b->nets.size(); ++k) {
    if (only >= 0 && (int)k != only) continue;
    BNet &N = b->nets[k].d;
    const size_t st = (size_t)N.B * N.ldl * 4;
    float *arrs[] = {N.mu_p, N.mu_m, N.v_p, N.v_m, N.s_p, N.s_m};
    for (float *a : arrs)
      if (e == hipSuccess) e = hipMemsetAsync(a, 0, st, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(N.V_hi, 0, (size_t)N.Bp * N.ldl * 2, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(N.V_lo, 0, (size_t)N.Bp * N.ldl * 2, b->stream);
    double *d8[] = {N.lam, N.vlam, N.slam};
    for (double *a : d8)
      if (e == hipSuccess) e = hipMemsetAsync(a, 0, (size_t)2 * N.B * 8, b->stream);
    if (e == hipSuccess)
      e = hipMemsetAsync(N.unitpart, 0, (size_t)2 * N.ncb * N.Bp * 2 * 8, b->stream);
  }
  // the other networks keep their state; it moves to the slot that
  // iteration k0 reads
  if (only >= 0 && ((b->iters ^ k0) & 1)) {
    const int from = (int)(b->iters & 1), to = (int)(k0 & 1);
    for (size_t k = 0; k < b->nets.size(); ++k) {
      if ((int)k == only) continue;
      const BNet &N = b->nets[k].d;
      double *d8[] = {N.lam, N.vlam, N.slam};
      for (double *a : d8)
        if (e == hipSuccess)
          e = hipMemcpyAsync(a + (size_t)to * N.B, a + (size_t)from * N.B, (size_t)N.B * 8,
                             hipMemcpyDeviceToDevice, b->stream);
    }
  }
  BScal s{};
  s.it[k0 & 1].k = k0;
  s.it[k0 & 1].pending = 0;
  s.it[(k0 + 1) & 1].k = k0 + 1;
  if (e == hipSuccess) e = hipMemcpyAsync(b->sc, &s, sizeof(s), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  b->iters = k0;
  return e;
}

hipError_t upload_nets(dcopf_batch_s *b) {
  std::vector<BNet> h(b->nets.size());
  for (size_t k = 0; k < h.size(); ++k) h[k] = b->nets[k].d;
  return hipMemcpy(b->d_nets, h.data(), h.size() * sizeof(BNet), hipMemcpyHostToDevice);
}

hipError_t upload_tables(dcopf_batch_s *b) {
  std::vector<int> all(b->nets.size());
  std::iota(all.begin(), all.end(), 0);
  std::vector<int4> wt, ft;
  build_tables(b->nets, all, &wt, &ft);
  b->pool.put(b->d_wtiles);
  b->pool.put(b->d_ftiles);
  b->d_wtiles = b->d_ftiles = nullptr;
  b->d_wtiles = b->d_ftiles = nullptr;
  b->d_wtiles = b->pool.get_n<int4>(std::max<size_t>(1, wt.size()));
  b->d_ftiles = b->pool.get_n<int4>(std::max<size_t>(1, ft.size()));
  hipError_t e = (b->d_wtiles && b->d_ftiles) ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess)
    e = hipMemcpy(b->d_wtiles, wt.data(), wt.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_ftiles, ft.data(), ft.size() * sizeof(int4), hipMemcpyHostToDevice);
  b->n_wtiles = (int)wt.size();
  b->n_ftiles = (int)ft.size();
  return e;
}

// time `reps` launches of one phase for network k alone (ms per launch)
// (Re)capture graph_iters iterations (an even count, so the parity slots
// line up on every replay) as one HIP graph; the tile tables are baked in.
hipError_t capture_graph(dcopf_batch_s *b) {
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->graph_exec = nullptr;
  b->graph = nullptr;
  if (b->graph_iters <= 0) return hipSuccess;
  hipStream_t cs = nullptr;
  hipError_t ce = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (ce == hipSuccess) ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (ce == hipSuccess) {
    launch_iters_b(b, cs, 0, b->graph_iters);
    ce = hipStreamEndCapture(cs, &b->graph);
  }
  if (ce == hipSuccess) ce = hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  return ce;
}

// average ms of one whole iteration (every network, the three launches);
// the best of three runs of `reps` iterations
float time_iters(dcopf_batch_s *b, int reps) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1e30f;
  launch_iters_b(b, b->stream, b->iters, 2);
  b->iters += 2;
  float best = 1e30f;
  for (int trial = 0; trial < 3; ++trial) {
    (void)hipEventRecord(e0, b->stream);
    launch_iters_b(b, b->stream, b->iters, reps);
    b->iters += reps;
    (void)hipEventRecord(e1, b->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, ms / reps);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// Coordinate search over the tile shape and K split of the W product and
// the tile shape of the F product, one network at a time with the others
// fixed, timing whole iterations of the full batch (so tail effects of the
// shared launches count).  A candidate replaces the incumbent only when it
// is at least 2 % faster, which keeps the choice stable against timing noise.
// The iterate is disturbed; the caller resets it.  Each timing is the best
// of three runs of kTuneReps iterations (shorter runs let timing noise pick
// a slower W tile for the 10,000-bus network now and then).
constexpr int kTuneReps = 20;
hipError_t autotune(dcopf_batch_s *b) {
  const int splits[] = {1, 2, 4, 8, 16, 32};
  auto apply = [&]() -> hipError_t {
    hipError_t e = upload_nets(b);
    if (e == hipSuccess) e = upload_tables(b);
    return e;
  };
  std::vector<int> req_split(b->nets.size());
  for (size_t k = 0; k < b->nets.size(); ++k) req_split[k] = b->nets[k].d.S;
  hipError_t e = apply();
  if (e != hipSuccess) return e;
  float best = time_iters(b, kTuneReps);
  for (int sweep = 0; sweep < 2; ++sweep) {
    for (size_t k = 0; k < b->nets.size(); ++k) {
      BNet &N = b->nets[k].d;
      // tile shapes whose M extent exceeds the instances (rounded up to 32)
      // only multiply padding: not candidates
      auto fits = [&](int c) { return kTileBM[c] <= (N.B + 31) / 32 * 32; };
      int bw = N.cfg_w, bs = req_split[k];
      for (int c = 0; c < 3; ++c)
        for (int S : splits) {
          if (!fits(c)) continue;
          if (S > 1 && N.ldl / S < 256) continue;
          if (c == bw && S == bs) continue;
          N.cfg_w = c;
          set_split(N, S);
          if ((e = apply()) != hipSuccess) return e;
          const float t = time_iters(b, kTuneReps);
          if (t < 0.98f * best) best = t, bw = c, bs = S;
        }
      N.cfg_w = bw;
      set_split(N, bs);
      req_split[k] = bs;
      int bf = N.cfg_f;
      for (int c = 0; c < 3; ++c) {
        if (c == bf || !fits(c)) continue;
        N.cfg_f = c;
        if ((e = apply()) != hipSuccess) return e;
        const float t = time_iters(b, kTuneReps);
        if (t < 0.98f * best) best = t, bf = c;
      }
      N.cfg_f = bf;
      if ((e = apply()) != hipSuccess) return e;
    }
  }
  return apply();
}

dcopf_status validate_net(const dcopf_batch_network &n, int idx, size_t inst0) {
  const std::string tag = "network " + std::to_string(idx) + ": ";
  if (n.n_bus < 2 || n.n_line < 1 || n.n_gen < 1 || n.n_inst < 1)
    return set_error(tag + "need n_bus >= 2, n_line, n_gen, n_inst >= 1"), DCOPF_E_INVALID;
  if (n.n_line > (1 << 20) || n.n_bus > (1 << 24) || n.n_inst > (1 << 16))
    return set_error(tag + "too large"), DCOPF_E_INVALID;
  if (n.slack < 0 || n.slack >= n.n_bus) return set_error(tag + "slack out of range"), DCOPF_E_INVALID;
  if (!n.H || !n.gen_bus || !n.p_min || !n.p_max || !n.f_max || !n.d || !n.c)
    return set_error(tag + "null data pointer"), DCOPF_E_INVALID;
  const size_t nl = n.n_line, nb = n.n_bus, ng = n.n_gen, B = n.n_inst;
  if ((double)nl * (double)nb > 4.0e9) return set_error(tag + "H too large"), DCOPF_E_INVALID;
  // line-state arrays are addressed with 32-bit byte offsets
  if ((B + 127) / 128 * 128 * ((nl + 127) / 128 * 128) >= ((size_t)1 << 30))
    return set_error(tag + "n_inst * n_line too large (split the instances)"), DCOPF_E_INVALID;
  for (size_t g = 0; g < ng; ++g)
    if (n.gen_bus[g] < 0 || n.gen_bus[g] >= n.n_bus)
      return set_error(tag + "gen_bus out of range"), DCOPF_E_INVALID;
  if (!finite_all_b(n.H, nl * nb)) return set_error(tag + "H not finite"), DCOPF_E_INVALID;
  if (!finite_all_b(n.p_min, ng) || !finite_all_b(n.p_max, ng) || !finite_all_b(n.f_max, nl) ||
      !finite_all_b(n.d, B * nb) || !finite_all_b(n.c, B * ng) ||
      (n.q && !finite_all_b(n.q, B * ng)))
    return set_error(tag + "non-finite data"), DCOPF_E_INVALID;
  for (size_t g = 0; g < ng; ++g)
    if (n.p_min[g] > n.p_max[g]) return set_error(tag + "p_min > p_max"), DCOPF_E_INVALID;
  if (n.q)
    for (size_t t = 0; t < B * ng; ++t)
      if (n.q[t] < 0) return set_error(tag + "q < 0"), DCOPF_E_INVALID;
  for (size_t l = 0; l < nl; ++l)
    if (!(n.f_max[l] > 0)) return set_error(tag + "f_max <= 0"), DCOPF_E_INVALID;
  for (size_t l = 0; l < nl; ++l)
    if (n.H[l * nb + n.slack] != 0.0)
      return set_error(tag + "H column of the slack bus is not zero"), DCOPF_E_INVALID;
  if (!(n.alpha > 0) || !std::isfinite(n.alpha) || !(n.rho >= 0 && n.rho < 1))
    return set_error(tag + "alpha must be > 0 and rho in [0,1)"), DCOPF_E_INVALID;
  double smin = 0, smax = 0;
  for (size_t g = 0; g < ng; ++g) smin += n.p_min[g], smax += n.p_max[g];
  for (size_t i = 0; i < B; ++i) {
    double D = 0;
    for (size_t bb = 0; bb < nb; ++bb) D += n.d[i * nb + bb];
    if (D < smin - 1e-9 * std::max(1.0, std::fabs(D)) ||
        D > smax + 1e-9 * std::max(1.0, std::fabs(D)))
      return set_error(tag + "instance " + std::to_string(inst0 + i) +
                       ": total load outside [sum p_min, sum p_max]"),
             DCOPF_E_INFEASIBLE;
  }
  return DCOPF_OK;
}

dcopf_status setup_net(dcopf_batch_s *b, HostNet &hn, const dcopf_batch_network &n, int inst0) {
  BNet &N = hn.d;
  DevPool &own = b->pool;
  bool ok = true;
  const int nb = n.n_bus, nl = n.n_line, ng = n.n_gen, B = n.n_inst;
  std::vector<int> cols(n.gen_bus, n.gen_bus + ng);
  std::sort(cols.begin(), cols.end());
  cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  const int nc = (int)cols.size();
  std::vector<int> col_of_bus(nb, -1);
  for (int j = 0; j < nc; ++j) col_of_bus[cols[j]] = j;
  std::vector<int> gperm(ng);
  std::iota(gperm.begin(), gperm.end(), 0);
  std::stable_sort(gperm.begin(), gperm.end(), [&](int a, int c) {
    return col_of_bus[n.gen_bus[a]] < col_of_bus[n.gen_bus[c]];
  });
  std::vector<int> seg(nc + 1, 0);
  for (int g = 0; g < ng; ++g) seg[col_of_bus[n.gen_bus[g]] + 1]++;
  for (int j = 0; j < nc; ++j) seg[j + 1] += seg[j];
  std::vector<int> ucol(ng);
  for (int j = 0; j < nc; ++j)
    for (int u = seg[j]; u < seg[j + 1]; ++u) ucol[u] = j;
  hn.n_bus = nb;
  hn.gperm = gperm;
  hn.seg = seg;
  N.n_l = nl;
  N.n_c = nc;
  N.n_g = ng;
  N.B = B;
  N.Bp = (int)round_up(B, 128);  // every tile shape divides the padded extents
  N.ldl = (int)round_up(nl, 64);
  N.ldc = (int)round_up(nc, 64);
  N.ncp = (int)round_up(nc, 128);
  N.nlp = (int)round_up(nl, 128);
  N.ntl = (nl + 31) / 32;  // 32-line tiles carrying line terms
  N.inst0 = inst0;
  N.alpha = n.alpha;
  N.rho = n.rho;
  // default shapes: tall tiles when there are many instances, wide otherwise
  N.cfg_w = B >= 128 ? 0 : (B > 32 ? 1 : 2);
  N.cfg_f = N.cfg_w;
  // a network whose split panels (both orientations) would take most of the
  // last-level cache streams them nontemporally, leaving the cache to the
  // other networks' panels and the line state
  N.nt_panel = (double)4 * 2 * (double)nl * (double)nc >= kNtPanelBytes ? 1 : 0;
  set_split(N, N.Bp >= 256 ? 1 : std::max(1, N.ldl / 2048));
  const size_t Bp = N.Bp, ldl = N.ldl, ldc = N.ldc, ncp = N.ncp, nlp = N.nlp;
  __bf16 *PT_hi = balloc<__bf16>(own, ncp * ldl, &ok), *PT_lo = balloc<__bf16>(own, ncp * ldl, &ok);
  __bf16 *P_hi = balloc<__bf16>(own, nlp * ldc, &ok), *P_lo = balloc<__bf16>(own, nlp * ldc, &ok);
  double *P64T = balloc<double>(own, ncp * ldl, &ok);
  N.V_hi = balloc<__bf16>(own, Bp * ldl, &ok);
  N.V_lo = balloc<__bf16>(own, Bp * ldl, &ok);
  N.X_hi = balloc<__bf16>(own, Bp * ldc, &ok);
  N.X_lo = balloc<__bf16>(own, Bp * ldc, &ok);
  N.Wws = balloc<float>(own, (size_t)32 * Bp * ncp, &ok);
  float **st[] = {&N.mu_p, &N.mu_m, &N.v_p, &N.v_m, &N.s_p, &N.s_m};
  for (float **a : st) *a = balloc<float>(own, (size_t)B * ldl, &ok);
  float *fd32 = balloc<float>(own, (size_t)B * ldl, &ok);
  float *fl32 = balloc<float>(own, nl, &ok);
  double *fl64 = balloc<double>(own, nl, &ok);
  double *fd64 = balloc<double>(own, (size_t)B * nl, &ok);
  double *c = balloc<double>(own, (size_t)B * ng, &ok), *q = balloc<double>(own, (size_t)B * ng, &ok);
  double *pmin = balloc<double>(own, ng, &ok), *pmax = balloc<double>(own, ng, &ok);
  int *dseg = balloc<int>(own, nc + 1, &ok);
  int *ducol = balloc<int>(own, ng, &ok);
  N.lam = balloc<double>(own, (size_t)2 * B, &ok);
  N.vlam = balloc<double>(own, (size_t)2 * B, &ok);
  N.slam = balloc<double>(own, (size_t)2 * B, &ok);
  N.ncb = (nc + kUnitCols - 1) / kUnitCols;
  N.unitpart = balloc<double>(own, (size_t)2 * N.ncb * Bp * 2, &ok);
  double *D = balloc<double>(own, B, &ok);
  N.linepart = balloc<double>(own, (size_t)(nlp / 32) * Bp, &ok);  // every 32-line tile an F tile can write
  N.V64 = balloc<double>(own, Bp * ldl, &ok);
  N.W64 = balloc<double>(own, Bp * ncp, &ok);
  N.bound = balloc<double>(own, B, &ok);
  N.psum = balloc<double>(own, (size_t)B * ng, &ok);
  N.pbar = balloc<double>(own, (size_t)B * ng, &ok);
  N.P64 = balloc<double>(own, nlp * ldc, &ok);
  N.X64 = balloc<double>(own, Bp * ldc, &ok);
  N.F64 = balloc<double>(own, Bp * nlp, &ok);
  N.ppart = balloc<double>(own, (size_t)B * (2 * kPrimalColBlocks + 5), &ok);
  if (!ok) return set_error("device allocation failed"), DCOPF_E_NOMEM;
  N.PT_hi = PT_hi;
  N.PT_lo = PT_lo;
  N.P_hi = P_hi;
  N.P_lo = P_lo;
  N.P64T = P64T;
  N.fd32 = fd32;
  N.flim32 = fl32;
  N.flim64 = fl64;
  N.fd64 = fd64;
  N.c = c;
  N.q = q;
  N.pmin = pmin;
  N.pmax = pmax;
  N.seg = dseg;
  N.ucol = ducol;
  N.D = D;
  hipStream_t s = b->stream;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (r != hipSuccess && e == hipSuccess) e = r;
  };
  // temporaries: H (padded rows for the f_d product), loads, gathered panel
  const size_t ldb = (size_t)round_up(nb, 4), nlp16 = (size_t)round_up(nl, 16);
  double *Hd = nullptr, *Dm = nullptr, *tmp = nullptr, *fdt = nullptr;
  int *dcols = nullptr;
  Hd = b->pool.get_n<double>(nlp16 * ldb);
  Dm = b->pool.get_n<double>(Bp * ldb);
  tmp = b->pool.get_n<double>(nlp * ldc);
  fdt = b->pool.get_n<double>(Bp * nlp16);
  dcols = b->pool.get_n<int>((size_t)nc);
  if (!Hd || !Dm || !tmp || !fdt || !dcols) chk(hipErrorOutOfMemory);
  if (e == hipSuccess) {
    chk(hipMemsetAsync(Hd, 0, nlp16 * ldb * 8, s));
    chk(hipMemcpy2DAsync(Hd, ldb * 8, n.H, (size_t)nb * 8, (size_t)nb * 8, nl,
                         hipMemcpyHostToDevice, s));
    chk(hipMemsetAsync(Dm, 0, Bp * ldb * 8, s));
    chk(hipMemcpy2DAsync(Dm, ldb * 8, n.d, (size_t)nb * 8, (size_t)nb * 8, B,
                         hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(dcols, cols.data(), (size_t)nc * 4, hipMemcpyHostToDevice, s));
    // panel: gather, split; transpose to FP64 P^T, split
    dim3 gg((unsigned)std::min<size_t>(64, (ldc + 255) / 256), (unsigned)nlp);
    bgather_kernel<<<gg, 256, 0, s>>>(Hd, (int)ldb, nl, dcols, nc, (int)ldc, tmp);
    chk(hipMemcpyAsync(N.P64, tmp, nlp * ldc * 8, hipMemcpyDeviceToDevice, s));
    bsplit_kernel<<<2048, 256, 0, s>>>(tmp, nlp * ldc, P_hi, P_lo);
    dim3 tg((unsigned)(ncp / 32), (unsigned)(ldl / 32));
    btranspose_kernel<<<tg, dim3(32, 8), 0, s>>>(tmp, nl, (int)ldc, (int)ncp, (int)ldl, P64T);
    bsplit_kernel<<<2048, 256, 0, s>>>(P64T, ncp * ldl, PT_hi, PT_lo);
    // f_d = H d for every instance (FP64 matrix cores)
    dim3 dg((unsigned)(nlp16 / 16), (unsigned)(Bp / 64));
    dgemm_nt_kernel<<<dg, 256, 0, s>>>(Dm, Hd, fdt, (int)ldb, (int)nlp16, (int)Bp);
    dim3 fg((unsigned)std::min<size_t>(64, (nl + 255) / 256), (unsigned)B);
    chk(hipMemsetAsync(fd32, 0, (size_t)B * ldl * 4, s));
    bfd_kernel<<<fg, 256, 0, s>>>(fdt, (int)nlp16, B, nl, (int)ldl, fd64, fd32);
    chk(hipGetLastError());
    // data
    std::vector<float> f32(n.f_max, n.f_max + nl);
    // unit data in column-sorted order: unit t of the panel is generator gperm[t]
    std::vector<double> cs((size_t)B * ng), qs((size_t)B * ng, 0.0), lo(ng), hi(ng), Dh(B, 0.0);
    for (int t = 0; t < ng; ++t) {
      const int g = gperm[t];
      lo[t] = n.p_min[g];
      hi[t] = n.p_max[g];
      for (int i = 0; i < B; ++i) {
        cs[(size_t)i * ng + t] = n.c[(size_t)i * ng + g];
        if (n.q) qs[(size_t)i * ng + t] = n.q[(size_t)i * ng + g];
      }
    }
    for (int i = 0; i < B; ++i)
      for (int bb = 0; bb < nb; ++bb) Dh[i] += n.d[(size_t)i * nb + bb];
    chk(hipMemcpyAsync(fl32, f32.data(), nl * 4, hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(fl64, n.f_max, nl * 8, hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(c, cs.data(), (size_t)B * ng * 8, hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(q, qs.data(), (size_t)B * ng * 8, hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(pmin, lo.data(), ng * 8, hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(pmax, hi.data(), ng * 8, hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(dseg, seg.data(), (nc + 1) * 4, hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(ducol, ucol.data(), (size_t)ng * 4, hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(D, Dh.data(), B * 8, hipMemcpyHostToDevice, s));
    chk(hipMemsetAsync(N.X_hi, 0, Bp * ldc * 2, s));
    chk(hipMemsetAsync(N.X_lo, 0, Bp * ldc * 2, s));
    chk(hipMemsetAsync(N.V64, 0, Bp * ldl * 8, s));
    chk(hipMemsetAsync(N.linepart, 0, (size_t)(nlp / 32) * Bp * 8, s));
    chk(hipMemsetAsync(N.psum, 0, (size_t)B * ng * 8, s));
    chk(hipMemsetAsync(N.X64, 0, Bp * ldc * 8, s));
    chk(hipStreamSynchronize(s));
  }
  b->pool.put(Hd);
  b->pool.put(Dm);
  b->pool.put(tmp);
  b->pool.put(fdt);
  b->pool.put(dcols);
  if (e != hipSuccess)
    return set_error(std::string("HIP error in batch setup: ") + hipGetErrorString(e)),
           DCOPF_E_HIP;
  return DCOPF_OK;
}

dcopf_status eval_bounds(dcopf_batch_s *b) {
  hipStream_t s = b->stream;
  for (auto &hn : b->nets) {
    const BNet &N = hn.d;
    dim3 vg((unsigned)std::min(64, (N.n_l + 255) / 256), (unsigned)N.B);
    make_v64_kernel<<<vg, 256, 0, s>>>(N.mu_p, N.mu_m, N.B, N.n_l, N.ldl, N.V64);
    dim3 dg((unsigned)(N.ncp / 16), (unsigned)(N.Bp / 64));
    dgemm_nt_kernel<<<dg, 256, 0, s>>>(N.V64, N.P64T, N.W64, N.ldl, N.ncp, N.Bp);
    bound_inst_kernel<<<N.B, 256, 0, s>>>(N, (int)(b->iters & 1));
  }
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(s));
  return DCOPF_OK;
}

}  // namespace

extern "C" {

dcopf_status dcopf_batch_create(const dcopf_batch_network *nets, int32_t n_nets,
                                const dcopf_batch_opts *opts, void *hip_stream,
                                dcopf_batch_t *out) {
  if (!out) return set_error("out is NULL"), DCOPF_E_INVALID;
  *out = nullptr;
  set_error("");
  if (!nets || n_nets < 1 || n_nets > 64 || !opts)
    return set_error("need 1..64 networks and options"), DCOPF_E_INVALID;
  const dcopf_batch_opts &o = *opts;
  if (o.rule < 0 || o.rule > 2) return set_error("unknown rule"), DCOPF_E_INVALID;
  if (o.rule == DCOPF_RULE_ADAM &&
      !(o.beta1 >= 0 && o.beta1 < 1 && o.beta2 >= 0 && o.beta2 < 1))
    return set_error("beta1, beta2 must be in [0,1)"), DCOPF_E_INVALID;
  if (o.rule != DCOPF_RULE_GDM && !(o.eps > 0)) return set_error("eps must be > 0"), DCOPF_E_INVALID;
  if (!(o.decay >= 0) || !std::isfinite(o.decay)) return set_error("decay must be >= 0"), DCOPF_E_INVALID;
  if (o.graph_iters < 0 || o.graph_iters > 4096)
    return set_error("graph_iters must be in [0, 4096]"), DCOPF_E_INVALID;
  if (o.gamma_cap < 1 || o.gamma_cap > 65536 || (o.gamma_cap & (o.gamma_cap - 1)))
    return set_error("gamma_cap must be a power of two in [1, 65536]"), DCOPF_E_INVALID;
  size_t total = 0;
  for (int k = 0; k < n_nets; ++k) {
    dcopf_status st = validate_net(nets[k], k, total);
    if (st != DCOPF_OK) return st;
    total += nets[k].n_inst;
  }
  if (total > (1u << 20)) return set_error("too many instances"), DCOPF_E_INVALID;
  auto *b = new dcopf_batch_s();
  b->opts = o;
  b->prm = BParams{o.rule, o.literal, o.beta1, o.beta2, o.eps, o.decay};
  b->stream = (hipStream_t)hip_stream;
  b->pool.mem = current_devmem(hip_stream);
  b->nets.resize(n_nets);
  b->n_total = (int)total;
  int inst0 = 0;
  for (int k = 0; k < n_nets; ++k) {
    dcopf_status st = setup_net(b, b->nets[k], nets[k], inst0);
    if (st != DCOPF_OK) {
      free_batch(b);
      return st;
    }
    inst0 += nets[k].n_inst;
  }
  std::vector<int2> inst;
  std::vector<int4> units;
  for (int k = 0; k < n_nets; ++k)
    for (int i = 0; i < nets[k].n_inst; ++i) {
      inst.push_back(make_int2(k, i));
      for (int cb = 0; cb < b->nets[k].d.ncb; ++cb) {
        // network and column block packed (k < 64, cb < 2^15), the block's units
        const int jb = cb * kUnitCols, je = std::min(b->nets[k].d.n_c, jb + kUnitCols);
        units.push_back(make_int4(k | (cb << 16), i, b->nets[k].seg[jb], b->nets[k].seg[je]));
      }
    }
  b->n_units = (int)units.size();
  b->gcap = o.gamma_cap;
  b->d_nets = b->pool.get_n<BNet>(n_nets);
  b->d_inst = b->pool.get_n<int2>(inst.size());
  b->d_units = b->pool.get_n<int4>(units.size());
  hipError_t e = (b->d_nets && b->d_inst && b->d_units) ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess)
    e = hipMemcpy(b->d_units, units.data(), units.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    b->sc = b->pool.get_n<BScal>(1);
    b->gam = b->pool.get_n<double>((size_t)b->gcap * total);
    if (!b->sc || !b->gam) e = hipErrorOutOfMemory;
  }
  if (e == hipSuccess)
    e = hipMemcpy(b->d_inst, inst.data(), inst.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(b->gam, 0, (size_t)b->gcap * total * 8);
  if (e == hipSuccess) e = upload_nets(b);
  if (e == hipSuccess) e = reset_state(b, 0);
  if (e == hipSuccess && o.autotune) e = autotune(b);
  if (e == hipSuccess) e = upload_tables(b);
  if (e == hipSuccess) e = reset_state(b, 0);
  if (e != hipSuccess) {
    set_error(std::string("HIP error in batch create: ") + hipGetErrorString(e));
    free_batch(b);
    return DCOPF_E_HIP;
  }
  b->best.assign(total, -INFINITY);
  b->best_iter.assign(total, -1);
  b->graph_iters = (o.graph_iters + 1) / 2 * 2;
  hipError_t ce = capture_graph(b);
  if (ce != hipSuccess) {
    set_error(std::string("graph capture failed: ") + hipGetErrorString(ce));
    free_batch(b);
    return DCOPF_E_HIP;
  }
  *out = b;
  return DCOPF_OK;
}

dcopf_status dcopf_batch_step(dcopf_batch_t b, int64_t n) {
  if (!b || n < 0) return set_error("null handle or n < 0"), DCOPF_E_INVALID;
  if (n == 0) return DCOPF_OK;
  int64_t left = n;
  if (b->graph_exec) {
    if (b->iters & 1) {
      launch_iters_b(b, b->stream, b->iters, 1);
      b->iters += 1;
      left -= 1;
    }
    while (left >= b->graph_iters) {
      DCOPF_HIP_TRY(hipGraphLaunch(b->graph_exec, b->stream));
      b->iters += b->graph_iters;
      left -= b->graph_iters;
    }
  }
  launch_iters_b(b, b->stream, b->iters, left);
  b->iters += left;
  launch_final_b(b, b->stream);
  DCOPF_HIP_TRY(hipGetLastError());
  return DCOPF_OK;
}

dcopf_status dcopf_batch_bound(dcopf_batch_t b, double *values) {
  if (!b || !values) return set_error("null argument"), DCOPF_E_INVALID;
  dcopf_status st = eval_bounds(b);
  if (st != DCOPF_OK) return st;
  bool finite = true;
  for (auto &hn : b->nets) {
    const BNet &N = hn.d;
    DCOPF_HIP_TRY(hipMemcpy(values + N.inst0, N.bound, (size_t)N.B * 8, hipMemcpyDeviceToHost));
  }
  for (int i = 0; i < b->n_total; ++i) {
    if (!std::isfinite(values[i])) finite = false;
    if (values[i] > b->best[i]) {
      b->best[i] = values[i];
      b->best_iter[i] = b->iters;
    }
  }
  if (!finite) return set_error("non-finite dual value"), DCOPF_E_NONFINITE;
  return DCOPF_OK;
}

dcopf_status dcopf_batch_best(dcopf_batch_t b, double *values, int64_t *iters) {
  if (!b) return set_error("null handle"), DCOPF_E_INVALID;
  for (int i = 0; i < b->n_total; ++i) {
    if (values) values[i] = b->best[i];
    if (iters) iters[i] = b->best_iter[i];
  }
  return DCOPF_OK;
}

dcopf_status dcopf_batch_solve(dcopf_batch_t b, const double *opt, double gap_tol,
                               int64_t max_iters, int64_t check_every, int64_t *first_hit) {
  if (!b || !opt || max_iters < 0 || check_every < 1)
    return set_error("bad arguments"), DCOPF_E_INVALID;
  std::vector<double> vals(b->n_total);
  std::vector<int64_t> hit(b->n_total, -1);
  int64_t done = 0;
  dcopf_status st = dcopf_batch_bound(b, vals.data());
  if (st != DCOPF_OK) return st;
  while (true) {
    int open = 0;
    for (int i = 0; i < b->n_total; ++i) {
      if (hit[i] < 0 && opt[i] - b->best[i] <= gap_tol * std::fabs(opt[i])) hit[i] = b->best_iter[i];
      if (hit[i] < 0) ++open;
    }
    if (open == 0 || done >= max_iters) break;
    const int64_t n = std::min<int64_t>(check_every, max_iters - done);
    st = dcopf_batch_step(b, n);
    if (st != DCOPF_OK) return st;
    done += n;
    st = dcopf_batch_bound(b, vals.data());
    if (st != DCOPF_OK) return st;
  }
  if (first_hit) std::copy(hit.begin(), hit.end(), first_hit);
  return DCOPF_OK;
}

dcopf_status dcopf_batch_gammas(dcopf_batch_t b, int64_t first, int64_t count, double *out) {
  if (!b || !out || first < 0 || count < 0) return set_error("bad arguments"), DCOPF_E_INVALID;
  if (first + count > b->iters || first < b->iters - b->gcap)
    return set_error("requested iterations not recorded"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  for (int64_t t = 0; t < count; ++t) {
    const int64_t k = (first + t) & (b->gcap - 1);
    DCOPF_HIP_TRY(hipMemcpy(out + t * b->n_total, b->gam + (size_t)k * b->n_total,
                            (size_t)b->n_total * 8, hipMemcpyDeviceToHost));
  }
  return DCOPF_OK;
}

dcopf_status dcopf_batch_get_multipliers(dcopf_batch_t b, int32_t net, double *lambda,
                                         double *mu_plus, double *mu_minus) {
  if (!b || net < 0 || net >= (int)b->nets.size()) return set_error("bad network"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  const BNet &N = b->nets[net].d;
  // after a step call the state of iteration `iters` sits in slot iters & 1
  if (lambda)
    DCOPF_HIP_TRY(hipMemcpy(lambda, N.lam + (size_t)(b->iters & 1) * N.B, (size_t)N.B * 8,
                            hipMemcpyDeviceToHost));
  std::vector<float> tmp((size_t)N.B * N.ldl);
  float *src[2] = {N.mu_p, N.mu_m};
  double *dst[2] = {mu_plus, mu_minus};
  for (int s = 0; s < 2; ++s) {
    if (!dst[s]) continue;
    DCOPF_HIP_TRY(hipMemcpy(tmp.data(), src[s], tmp.size() * 4, hipMemcpyDeviceToHost));
    for (int i = 0; i < N.B; ++i)
      for (int l = 0; l < N.n_l; ++l) dst[s][(size_t)i * N.n_l + l] = tmp[(size_t)i * N.ldl + l];
  }
  return DCOPF_OK;
}

dcopf_status dcopf_batch_set_multipliers(dcopf_batch_t b, int32_t net, const double *lambda,
                                         const double *mu_plus, const double *mu_minus) {
  if (!b || net < 0 || net >= (int)b->nets.size() || !lambda || !mu_plus || !mu_minus)
    return set_error("bad arguments"), DCOPF_E_INVALID;
  const BNet &N = b->nets[net].d;
  const size_t n = (size_t)N.B * N.n_l;
  if (!finite_all_b(lambda, N.B) || !finite_all_b(mu_plus, n) || !finite_all_b(mu_minus, n))
    return set_error("non-finite multipliers"), DCOPF_E_INVALID;
  for (size_t t = 0; t < n; ++t)
    if (mu_plus[t] < 0 || mu_minus[t] < 0) return set_error("mu must be >= 0"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  // this network's optimiser state restarts; the batch's iteration counter
  // (step decay, Adam bias correction) restarts at 0 for every network
  DCOPF_HIP_TRY(reset_state(b, 0, net));
  std::vector<float> tmp((size_t)N.B * N.ldl, 0.f);
  const double *srcs[2] = {mu_plus, mu_minus};
  float *dsts[2] = {N.mu_p, N.mu_m};
  for (int s = 0; s < 2; ++s) {
    for (int i = 0; i < N.B; ++i)
      for (int l = 0; l < N.n_l; ++l) tmp[(size_t)i * N.ldl + l] = (float)srcs[s][(size_t)i * N.n_l + l];
    DCOPF_HIP_TRY(hipMemcpy(dsts[s], tmp.data(), tmp.size() * 4, hipMemcpyHostToDevice));
  }
  DCOPF_HIP_TRY(hipMemcpy(N.lam, lambda, (size_t)N.B * 8, hipMemcpyHostToDevice));  // slot 0
  dim3 vg((unsigned)std::min(64, (N.n_l + 255) / 256), (unsigned)N.B);
  bmake_v_kernel<<<vg, 256, 0, b->stream>>>(N.mu_p, N.mu_m, N.B, N.n_l, N.ldl, N.V_hi, N.V_lo);
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  std::fill(b->best.begin(), b->best.end(), -INFINITY);
  std::fill(b->best_iter.begin(), b->best_iter.end(), -1);
  return DCOPF_OK;
}

size_t dcopf_batch_state_len(dcopf_batch_t b, int32_t net) {
  if (!b || net < 0 || net >= (int)b->nets.size()) return 0;
  const BNet &N = b->nets[net].d;
  return 1 + 3 * (size_t)N.B + 6 * (size_t)N.B * N.n_l;
}

dcopf_status dcopf_batch_get_state(dcopf_batch_t b, int32_t net, double *buf, size_t len) {
  if (!b || net < 0 || net >= (int)b->nets.size() || !buf)
    return set_error("bad arguments"), DCOPF_E_INVALID;
  if (len != dcopf_batch_state_len(b, net)) return set_error("state length mismatch"), DCOPF_E_STATE;
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  const BNet &N = b->nets[net].d;
  const size_t B = N.B, nl = N.n_l;
  buf[0] = (double)b->iters;
  // after a step call the state of iteration `iters` sits in slot iters & 1
  const size_t slot = (size_t)(b->iters & 1) * B;
  const double *d8[] = {N.lam, N.vlam, N.slam};
  for (int a = 0; a < 3; ++a)
    DCOPF_HIP_TRY(hipMemcpy(buf + 1 + a * B, d8[a] + slot, B * 8, hipMemcpyDeviceToHost));
  std::vector<float> tmp(B * N.ldl);
  const float *f4[] = {N.mu_p, N.mu_m, N.v_p, N.v_m, N.s_p, N.s_m};
  double *out = buf + 1 + 3 * B;
  for (int a = 0; a < 6; ++a, out += B * nl) {
    DCOPF_HIP_TRY(hipMemcpy(tmp.data(), f4[a], tmp.size() * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < B; ++i)
      for (size_t l = 0; l < nl; ++l) out[i * nl + l] = tmp[i * N.ldl + l];
  }
  return DCOPF_OK;
}

dcopf_status dcopf_batch_set_state(dcopf_batch_t b, int32_t net, const double *buf, size_t len) {
  if (!b || net < 0 || net >= (int)b->nets.size() || !buf)
    return set_error("bad arguments"), DCOPF_E_INVALID;
  if (len != dcopf_batch_state_len(b, net)) return set_error("state length mismatch"), DCOPF_E_STATE;
  if (!finite_all_b(buf, len)) return set_error("non-finite state"), DCOPF_E_INVALID;
  const BNet &N = b->nets[net].d;
  const size_t B = N.B, nl = N.n_l;
  const double *mu = buf + 1 + 3 * B;
  for (size_t t = 0; t < 2 * B * nl; ++t)
    if (mu[t] < 0) return set_error("mu must be >= 0"), DCOPF_E_INVALID;
  const double *sq = buf + 1 + 3 * B + 4 * B * nl;
  for (size_t t = 0; t < 2 * B * nl; ++t)
    if (sq[t] < 0) return set_error("second moments must be >= 0"), DCOPF_E_INVALID;
  for (size_t i = 0; i < B; ++i)
    if (buf[1 + 2 * B + i] < 0) return set_error("second moments must be >= 0"), DCOPF_E_INVALID;
  if (buf[0] < 0 || buf[0] != std::floor(buf[0]) || buf[0] > 1e15)
    return set_error("iteration must be a nonnegative integer"), DCOPF_E_INVALID;
  const long long k0 = (long long)buf[0];
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  // zero this network's state; the batch's counter becomes k0 (the other
  // networks keep their state, moved to the slot iteration k0 reads)
  DCOPF_HIP_TRY(reset_state(b, k0, net));
  const size_t slot = (size_t)(k0 & 1) * B;
  double *d8[] = {N.lam, N.vlam, N.slam};
  for (int a = 0; a < 3; ++a)
    DCOPF_HIP_TRY(hipMemcpy(d8[a] + slot, buf + 1 + a * B, B * 8, hipMemcpyHostToDevice));
  std::vector<float> tmp(B * N.ldl, 0.f);
  float *f4[] = {N.mu_p, N.mu_m, N.v_p, N.v_m, N.s_p, N.s_m};
  const double *in = buf + 1 + 3 * B;
  for (int a = 0; a < 6; ++a, in += B * nl) {
    for (size_t i = 0; i < B; ++i)
      for (size_t l = 0; l < nl; ++l) tmp[i * N.ldl + l] = (float)in[i * nl + l];
    DCOPF_HIP_TRY(hipMemcpy(f4[a], tmp.data(), tmp.size() * 4, hipMemcpyHostToDevice));
  }
  dim3 vg((unsigned)std::min(64, (N.n_l + 255) / 256), (unsigned)N.B);
  bmake_v_kernel<<<vg, 256, 0, b->stream>>>(N.mu_p, N.mu_m, N.B, N.n_l, N.ldl, N.V_hi, N.V_lo);
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  for (size_t i = 0; i < B; ++i) {
    b->best[N.inst0 + i] = -INFINITY;
    b->best_iter[N.inst0 + i] = -1;
  }
  return DCOPF_OK;
}

dcopf_status dcopf_batch_set_start_dev(dcopf_batch_t b, int32_t net, const float *Y,
                                       int32_t ld) {
  if (!b || net < 0 || net >= (int)b->nets.size() || !Y)
    return set_error("bad arguments"), DCOPF_E_INVALID;
  const BNet &N = b->nets[net].d;
  if (ld < 2 * N.n_l + 1) return set_error("ld must be >= 2 n_line + 1"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  DCOPF_HIP_TRY(reset_state(b, 0, net));
  int *bad = b->pool.get_n<int>(1);
  if (!bad) return set_error("set_start_dev: device allocation failed"), DCOPF_E_NOMEM;
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), b->stream);
  dim3 vg((unsigned)std::min(64, (N.ldl + 255) / 256), (unsigned)N.B);
  if (e == hipSuccess) {
    bset_start_kernel<<<vg, 256, 0, b->stream>>>(N, Y, ld, bad);
    bmake_v_kernel<<<vg, 256, 0, b->stream>>>(N.mu_p, N.mu_m, N.B, N.n_l, N.ldl, N.V_hi, N.V_lo);
    e = hipGetLastError();
  }
  int hbad = 0;
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = hipMemcpy(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost);
  b->pool.put(bad);
  if (e != hipSuccess)
    return set_error(std::string("set_start_dev: ") + hipGetErrorString(e)), DCOPF_E_HIP;
  std::fill(b->best.begin(), b->best.end(), -INFINITY);
  std::fill(b->best_iter.begin(), b->best_iter.end(), -1);
  if (hbad) return set_error("non-finite start values"), DCOPF_E_NONFINITE;
  return DCOPF_OK;
}

dcopf_status dcopf_batch_adopt_better(dcopf_batch_t dst, int32_t dnet, dcopf_batch_t src,
                                      int32_t snet, int32_t *kept) {
  if (!dst || !src || dst == src || dnet < 0 || dnet >= (int)dst->nets.size() || snet < 0 ||
      snet >= (int)src->nets.size())
    return set_error("adopt: bad arguments"), DCOPF_E_INVALID;
  const BNet &D = dst->nets[dnet].d, &S = src->nets[snet].d;
  if (D.B != S.B || D.n_l != S.n_l || D.n_c != S.n_c || D.n_g != S.n_g || D.ldl != S.ldl)
    return set_error("adopt: the two networks differ in shape"), DCOPF_E_INVALID;
  if (dst->iters != src->iters)
    return set_error("adopt: the two batches are at different iterations"), DCOPF_E_STATE;
  if (dst->prm.rule != src->prm.rule)
    return set_error("adopt: the two batches use different step rules"), DCOPF_E_INVALID;
  // the same instances: equal total loads, instance by instance
  {
    std::vector<double> a(D.B), c(S.B);
    DCOPF_HIP_TRY(hipMemcpy(a.data(), D.D, (size_t)D.B * 8, hipMemcpyDeviceToHost));
    DCOPF_HIP_TRY(hipMemcpy(c.data(), S.D, (size_t)S.B * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < D.B; ++i)
      if (a[i] != c[i]) return set_error("adopt: instance loads differ"), DCOPF_E_INVALID;
  }
  DCOPF_HIP_TRY(hipStreamSynchronize(src->stream));
  dcopf_status st = eval_bounds(src);
  if (st == DCOPF_OK) st = eval_bounds(dst);
  if (st != DCOPF_OK) return st;
  int *dk = dst->pool.get_n<int>((size_t)D.B);
  if (!dk) return set_error("adopt: device allocation failed"), DCOPF_E_NOMEM;
  dim3 g((unsigned)std::min(64, (D.ldl + 255) / 256), (unsigned)D.B);
  badopt_kernel<<<g, 256, 0, dst->stream>>>(D, S, (int)(dst->iters & 1), dk);
  std::vector<int> hk(D.B);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(dst->stream);
  if (e == hipSuccess) e = hipMemcpy(hk.data(), dk, (size_t)D.B * sizeof(int), hipMemcpyDeviceToHost);
  dst->pool.put(dk);
  if (e != hipSuccess) return set_error(std::string("adopt: ") + hipGetErrorString(e)), DCOPF_E_HIP;
  for (int i = 0; i < D.B; ++i) {
    if (hk[i]) {
      dst->best[D.inst0 + i] = src->best[S.inst0 + i];
      dst->best_iter[D.inst0 + i] = src->best_iter[S.inst0 + i];
    }
    if (kept) kept[i] = hk[i];
  }
  return DCOPF_OK;
}

dcopf_status dcopf_batch_average(dcopf_batch_t b, int32_t enable) {
  if (!b) return set_error("null handle"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  BScal h{};
  DCOPF_HIP_TRY(hipMemcpy(&h, b->sc, sizeof(h), hipMemcpyDeviceToHost));
  if (enable) {
    for (auto &hn : b->nets)
      DCOPF_HIP_TRY(hipMemset(hn.d.psum, 0, (size_t)hn.d.B * hn.d.n_g * 8));
    h.avg_count = 0;
  }
  h.avg_on = enable ? 1 : 0;
  DCOPF_HIP_TRY(hipMemcpy(b->sc, &h, sizeof(h), hipMemcpyHostToDevice));
  return DCOPF_OK;
}

dcopf_status dcopf_batch_primal(dcopf_batch_t b, int32_t net, dcopf_primal *out,
                                double *p_avg) {
  if (!b || !out || net < 0 || net >= (int)b->nets.size())
    return set_error("bad arguments"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  BScal h{};
  DCOPF_HIP_TRY(hipMemcpy(&h, b->sc, sizeof(h), hipMemcpyDeviceToHost));
  if (h.avg_count <= 0) return set_error("no iterations averaged"), DCOPF_E_STATE;
  const HostNet &hn = b->nets[net];
  const BNet &N = hn.d;
  hipStream_t s = b->stream;
  const int gc = std::max(1, std::min(kPrimalColBlocks, (N.ldc + 255) / 256));
  double *part = N.ppart, *res = N.ppart + (size_t)N.B * 2 * kPrimalColBlocks;
  bprimal_cols_kernel<<<dim3((unsigned)gc, (unsigned)N.B), 256, 0, s>>>(N, b->sc, part);
  dim3 dg((unsigned)(N.nlp / 16), (unsigned)(N.Bp / 64));
  dgemm_nt_kernel<<<dg, 256, 0, s>>>(N.X64, N.P64, N.F64, N.ldc, N.nlp, N.Bp);
  bprimal_inst_kernel<<<N.B, 256, 0, s>>>(N, b->sc, part, gc, res);
  DCOPF_HIP_TRY(hipGetLastError());
  std::vector<double> r((size_t)N.B * 5), pb;
  DCOPF_HIP_TRY(hipMemcpyAsync(r.data(), res, r.size() * 8, hipMemcpyDeviceToHost, s));
  if (p_avg) {
    pb.resize((size_t)N.B * N.n_g);
    DCOPF_HIP_TRY(hipMemcpyAsync(pb.data(), N.pbar, pb.size() * 8, hipMemcpyDeviceToHost, s));
  }
  DCOPF_HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < N.B; ++i) {
    out[i].cost = r[(size_t)i * 5];
    out[i].balance = r[(size_t)i * 5 + 1];
    out[i].max_overload = r[(size_t)i * 5 + 2];
    out[i].sum_overload = r[(size_t)i * 5 + 3];
    out[i].iterations = h.avg_count;
    out[i].n_overloaded = (int32_t)r[(size_t)i * 5 + 4];
    if (p_avg)
      for (int t = 0; t < N.n_g; ++t)
        p_avg[(size_t)i * N.n_g + hn.gperm[t]] = pb[(size_t)i * N.n_g + t];
  }
  return DCOPF_OK;
}

dcopf_status dcopf_batch_repair(dcopf_batch_t b, int32_t net, const double *p_in,
                                int32_t max_rounds, dcopf_repair *out, double *p_out) {
  if (!b || !out || net < 0 || net >= (int)b->nets.size() || max_rounds < 0)
    return set_error("bad arguments"), DCOPF_E_INVALID;
  HostNet &hn = b->nets[net];
  BNet &N = hn.d;
  const int B = N.B, ng = N.n_g, nl = N.n_l;
  if (p_in)
    for (size_t k = 0; k < (size_t)B * ng; ++k)
      if (!std::isfinite(p_in[k])) return set_error("p_in is not finite"), DCOPF_E_INVALID;
  const int gc = std::max(1, std::min(kPrimalColBlocks, (N.ldc + 255) / 256));
  auto &R = hn.rep;
  if (!R.ready) {
    bool ok = true;
    DevPool &own = b->pool;
    R.pin = balloc<double>(own, (size_t)B * ng, &ok);
    R.p = balloc<double>(own, (size_t)B * ng, &ok);
    R.p0c = balloc<double>(own, (size_t)B * ng, &ok);
    R.W = balloc<double>(own, (size_t)B * N.ldc, &ok);
    R.t = balloc<double>(own, (size_t)B * kBRepRows, &ok);
    R.y = balloc<double>(own, (size_t)B * kBRepRows, &ok);
    R.G = balloc<double>(own, (size_t)B * kBRepRows * kBRepRows, &ok);
    R.L = balloc<double>(own, (size_t)B * kBRepRows * kBRepRows, &ok);
    R.A = balloc<double>(own, (size_t)B * kBRepRows * N.ldc, &ok);
    R.part = balloc<double>(own, (size_t)B * gc * 2, &ok);
    R.out = balloc<double>(own, (size_t)B * 4, &ok);
    R.pos = balloc<int>(own, (size_t)B * nl, &ok);
    R.rows = balloc<int>(own, (size_t)B * kBRepRows, &ok);
    R.sgn = balloc<int>(own, (size_t)B * kBRepRows, &ok);
    R.st = balloc<BRepState>(own, (size_t)B, &ok);
    if (!ok) return set_error("device allocation failed"), DCOPF_E_NOMEM;
    R.ready = true;
  }
  hipStream_t s = b->stream;
  DCOPF_HIP_TRY(hipStreamSynchronize(s));
  const double *src = R.pin;
  if (p_in) {
    std::vector<double> pc((size_t)B * ng);  // unit t of the column order is generator gperm[t]
    for (int i = 0; i < B; ++i)
      for (int t = 0; t < ng; ++t) pc[(size_t)i * ng + t] = p_in[(size_t)i * ng + hn.gperm[t]];
    DCOPF_HIP_TRY(hipMemcpyAsync(R.pin, pc.data(), pc.size() * 8, hipMemcpyHostToDevice, s));
    DCOPF_HIP_TRY(hipStreamSynchronize(s));
  } else {
    BScal h{};
    DCOPF_HIP_TRY(hipMemcpy(&h, b->sc, sizeof(h), hipMemcpyDeviceToHost));
    if (h.avg_count <= 0) return set_error("no iterations averaged"), DCOPF_E_STATE;
    bprimal_cols_kernel<<<dim3((unsigned)gc, (unsigned)B), 256, 0, s>>>(N, b->sc, N.ppart);
    src = N.pbar;
  }
  const int gi = std::min(64, (std::max(ng, nl) + 255) / 256);
  brep_init_kernel<<<dim3((unsigned)gi, (unsigned)B), 256, 0, s>>>(N, src, R.p, R.p0c, R.pos,
                                                                   R.st);
  std::vector<BRepState> hs(B);
  const dim3 dg((unsigned)(N.nlp / 16), (unsigned)(N.Bp / 64));
  const int ccb = (N.ldc + 255) / 256;
  for (;;) {
    brep_cols_kernel<<<dim3((unsigned)gc, (unsigned)B), 256, 0, s>>>(N, R.p, R.W, R.part);
    dgemm_nt_kernel<<<dg, 256, 0, s>>>(N.X64, N.P64, N.F64, N.ldc, N.nlp, N.Bp);
    brep_active_kernel<<<B, 256, 0, s>>>(N, R.part, gc, max_rounds, R.pos, R.rows, R.sgn, R.t,
                                         R.st);
    DCOPF_HIP_TRY(hipGetLastError());
    DCOPF_HIP_TRY(hipMemcpyAsync(hs.data(), R.st, (size_t)B * sizeof(BRepState),
                                 hipMemcpyDeviceToHost, s));
    DCOPF_HIP_TRY(hipStreamSynchronize(s));
    int new_rows = 0, live = 0;
    long long pairs = 0;
    for (const BRepState &x : hs) {
      if (x.stop) continue;
      ++live;
      new_rows = std::max(new_rows, x.m - x.m_old);
      pairs = std::max(pairs, (long long)(x.m + 1) * (x.m + 2) / 2);
    }
    if (live == 0) break;
    if (new_rows > 0)
      brep_gather_kernel<<<dim3((unsigned)(ccb * new_rows), (unsigned)B), 256, 0, s>>>(
          N, R.rows, R.st, ccb, R.A);
    brep_gram_kernel<<<dim3((unsigned)((pairs + 3) / 4), (unsigned)B), 256, 0, s>>>(N, R.A, R.W,
                                                                                   R.st, R.G);
    brep_solve_kernel<<<B, 1024, 0, s>>>(R.G, R.t, R.sgn, R.L, R.y, R.st);
    brep_step_kernel<<<dim3((unsigned)((N.n_c + 255) / 256), (unsigned)B), 256, 0, s>>>(
        N, R.A, R.y, R.st, R.p);
  }
  brep_final_kernel<<<B, 256, 0, s>>>(N, R.part, gc, R.p, R.p0c, R.out);
  DCOPF_HIP_TRY(hipGetLastError());
  std::vector<double> r((size_t)B * 4), pb;
  DCOPF_HIP_TRY(hipMemcpyAsync(r.data(), R.out, r.size() * 8, hipMemcpyDeviceToHost, s));
  if (p_out) {
    pb.resize((size_t)B * ng);
    DCOPF_HIP_TRY(hipMemcpyAsync(pb.data(), R.p, pb.size() * 8, hipMemcpyDeviceToHost, s));
  }
  DCOPF_HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < B; ++i) {
    out[i].cost = r[(size_t)i * 4];
    out[i].balance = r[(size_t)i * 4 + 1];
    out[i].max_overload = std::max(0.0, r[(size_t)i * 4 + 2]);
    out[i].max_shift = r[(size_t)i * 4 + 3];
    out[i].feasible = hs[i].done ? 1 : 0;
    out[i].rounds = hs[i].rounds;
    out[i].n_active = hs[i].m;
    out[i].pad = 0;
    if (p_out)
      for (int t = 0; t < ng; ++t) p_out[(size_t)i * ng + hn.gperm[t]] = pb[(size_t)i * ng + t];
  }
  return DCOPF_OK;
}

dcopf_status dcopf_batch_info(dcopf_batch_t b, int32_t net, int32_t *cfg, int64_t *iters) {
  if (!b || net < 0 || net >= (int)b->nets.size()) return set_error("bad network"), DCOPF_E_INVALID;
  const BNet &N = b->nets[net].d;
  if (cfg) {
    cfg[0] = kTileBM[N.cfg_w];
    cfg[1] = kTileBN[N.cfg_w];
    cfg[2] = N.S;
    cfg[3] = kTileBM[N.cfg_f] * 1000 + kTileBN[N.cfg_f];
  }
  if (iters) *iters = b->iters;
  return DCOPF_OK;
}

dcopf_status dcopf_batch_set_tiles(dcopf_batch_t b, int32_t net, const int32_t *cfg) {
  if (!b || !cfg || net < 0 || net >= (int)b->nets.size())
    return set_error("bad arguments"), DCOPF_E_INVALID;
  auto code = [](int bm, int bn) {
    for (int c = 0; c < 3; ++c)
      if (kTileBM[c] == bm && kTileBN[c] == bn) return c;
    return -1;
  };
  const int cw = code(cfg[0], cfg[1]), cf = code(cfg[3] / 1000, cfg[3] % 1000);
  if (cw < 0 || cf < 0) return set_error("unsupported tile shape"), DCOPF_E_INVALID;
  if (cfg[2] < 1 || cfg[2] > kMaxSplit)
    return set_error("K split must be in [1, 32]"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  BNet &N = b->nets[net].d;
  N.cfg_w = cw;
  N.cfg_f = cf;
  set_split(N, cfg[2]);
  DCOPF_HIP_TRY(upload_nets(b));
  DCOPF_HIP_TRY(upload_tables(b));
  DCOPF_HIP_TRY(capture_graph(b));
  return DCOPF_OK;
}

dcopf_status dcopf_batch_time_phases(dcopf_batch_t b, int64_t n, double *ms_out) {
  if (!b || !ms_out || n < 1) return set_error("bad arguments"), DCOPF_E_INVALID;
  // real iterations, each dispatch timed by events attached to it
  std::vector<hipEvent_t> ev(6 * (size_t)n, nullptr);
  for (auto &e : ev) DCOPF_HIP_TRY(hipEventCreate(&e));
  for (int64_t t = 0; t < n; ++t) {
    const int par = (int)((b->iters + t) & 1);
    hipEvent_t *E = &ev[6 * t];
    launch_w(b, b->stream, b->d_wtiles, b->n_wtiles, par, E[0], E[1]);
    launch_u(b, b->stream, par, E[2], E[3]);
    launch_f(b, b->stream, b->d_ftiles, b->n_ftiles, par, E[4], E[5]);
  }
  b->iters += n;
  launch_final_b(b, b->stream);
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(b->stream));
  double acc[3] = {0, 0, 0};
  for (int64_t t = 0; t < n; ++t)
    for (int p = 0; p < 3; ++p) {
      float ms = 0.f;
      DCOPF_HIP_TRY(hipEventElapsedTime(&ms, ev[6 * t + 2 * p], ev[6 * t + 2 * p + 1]));
      acc[p] += ms;
    }
  for (auto &e : ev) (void)hipEventDestroy(e);
  for (int p = 0; p < 3; ++p) ms_out[p] = acc[p] / n;
  return DCOPF_OK;
}

void dcopf_batch_destroy(dcopf_batch_t b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
}

}  // extern "C"
