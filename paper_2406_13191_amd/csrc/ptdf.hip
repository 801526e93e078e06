// PTDF construction (Section 2): H_a[:, kept] = Omega E_r B_r^{-1} with
// B_r = E_r^T Omega E_r and a zero slack column, in FP64 on the matrix
// cores.  n = n_bus - 1 reduced buses, padded to N = 64 T (identity rows).
//
//   1. B_r, one thread per row, from the lines incident to its bus;
//   2. B_r = L L^T, right-looking by blocks of 64: the diagonal block is
//      factored by one wavefront, which also forms its inverse; the
//      panel below it is L_ik = A_ik L_kk^{-T}; block columns go in pairs,
//      the second taking the first's update alone, then the trailing lower
//      triangle takes A_ij -= L_i,[k,k+1] L_j,[k,k+1]^T (K = 128);
//   3. W = L^{-1} on the identity, block row by block row: W_i = L_ii^{-1} W_i
//      over the tiles left of the diagonal, then W_j -= L_ji W_i below, rows
//      likewise in pairs (K = 128 for the rows below a pair);
//   4. X = B_r^{-1} = W^T W (into the buffer that held L), lower block
//      triangle, then mirrored;
//   5. H[l][bus] = b_l (X[f][bus] - X[t][bus]) on the kept buses.
//
// Every product is a 64 x 64 output tile of one workgroup of four
// wavefronts; a wavefront holds 16 rows as four 16 x 16 accumulators of
// v_mfma_f64_16x16x4f64.  Operands are read from global memory (L2) through
// strides, so one routine serves the three layouts (A B^T, A B, A^T B); the
// products with K = 64 issue all their loads before the first matrix
// instruction.
#include "common.h"
#include "dcopf_ptdf.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

namespace dcopf {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 64;  // block size

constexpr size_t round_up_c(size_t v, size_t m) { return (v + m - 1) / m * m; }

__device__ __forceinline__ int reduced(int bus, int slack) {
  return bus == slack ? -1 : (bus < slack ? bus : bus - 1);
}

// Row r of B_r (r < n) from the incidence lists; rows r >= n are identity
// rows.  A is zero on entry.
__global__ void assemble_kernel(const int *__restrict__ start, const int *__restrict__ adj,
                                const int *__restrict__ fbus, const int *__restrict__ tbus,
                                const double *__restrict__ b, int slack, int n, int N,
                                double *__restrict__ A) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < N; r += gridDim.x * blockDim.x) {
    double *row = A + (size_t)r * N;
    if (r >= n) {
      row[r] = 1.0;
      continue;
    }
    const int bus = r < slack ? r : r + 1;
    double diag = 0.0;
    for (int e = start[bus]; e < start[bus + 1]; ++e) {
      const int l = adj[e];
      const int other = fbus[l] == bus ? tbus[l] : fbus[l];
      diag += b[l];
      const int o = reduced(other, slack);
      if (o >= 0) row[o] -= b[l];
    }
    row[r] = diag;
  }
}

// acc[t] += A(m0 + i, k) B(k, 16 t + j) over k in [k0, k1), i, j < 16, where
// A(i, k) = Ap[i sar + k sak] (Ap at the wavefront's first row) and
// B(k, c) = Bp[k sbk + c sbc] (Bp at the tile's first column).  Lane l
// supplies A(l % 16, k + l / 16) and B(k + l / 16, l % 16); register j of
// accumulator t holds row 4 j + l / 16, column 16 t + l % 16.  KFIX > 0
// fixes k1 - k0 = KFIX at compile time, so every load of the product can be
// issued before the first matrix instruction.
template <int KFIX>
__device__ __forceinline__ void mma16x64(const double *Ap, size_t sar, size_t sak,
                                         const double *Bp, size_t sbk, size_t sbc, int k0,
                                         int k1, f64x4 (&acc)[4]) {
  const int lane = threadIdx.x & 63, r = lane & 15, kk = lane >> 4;
  const double *a = Ap + (size_t)r * sar + (size_t)kk * sak;
  const double *bb = Bp + (size_t)kk * sbk + (size_t)r * sbc;
  if (KFIX > 0) {
    constexpr int Q = KFIX > 0 ? KFIX / 4 : 1;
    double av[Q], bv[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const size_t k = (size_t)(k0 + 4 * q);
      av[q] = a[k * sak];
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[q][t] = bb[k * sbk + (size_t)(16 * t) * sbc];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q][t], acc[t], 0, 0, 0);
    return;
  }
  for (int k = k0; k < k1; k += 4) {
    const double av = a[(size_t)k * sak];
    double bv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) bv[t] = bb[(size_t)k * sbk + (size_t)(16 * t) * sbc];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[t], acc[t], 0, 0, 0);
  }
}

// out[(m0 + row) ld + col] for the wavefront's 16 rows: mode 0 store,
// mode 1 subtract.
__device__ __forceinline__ void store16x64(double *out, size_t ld, const f64x4 (&acc)[4],
                                           int mode) {
  const int lane = threadIdx.x & 63, m0 = (threadIdx.x >> 6) * 16;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double *p = out + (size_t)(m0 + 4 * j + (lane >> 4)) * ld + 16 * t + (lane & 15);
      *p = mode == 0 ? acc[t][j] : *p - acc[t][j];
    }
}

// Diagonal block kb, one wavefront: lane i holds row i of the block in
// registers (both loops unrolled, so every index is a constant).  Step j
// takes the pivot from lane j through LDS, scales column j and updates the
// rows below with column j, broadcast through LDS.  L goes back to A (zeros
// above the diagonal) and to LDS; lane c then forms column c of Y = L^{-1}
// by forward substitution with the rows of L read from LDS, and Y goes to
// Yd[kb].  flag = 1 on a pivot that is not positive.
__global__ __launch_bounds__(64) void potrf_kernel(double *__restrict__ A, int N, int kb,
                                                   double *__restrict__ Yd, int *flag) {
  __shared__ double Ls[kT][kT + 1];
  __shared__ double colj[kT];
  __shared__ double piv;
  const int i = threadIdx.x;
  double *blk = A + (size_t)kb * kT * N + (size_t)kb * kT;
  for (int r = 0; r < kT; ++r) Ls[r][i] = blk[(size_t)r * N + i];  // rows, coalesced
  __syncthreads();
  double row[kT];
#pragma unroll
  for (int c = 0; c < kT; ++c) row[c] = Ls[i][c];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < kT; ++j) {
    if (i == j) piv = row[j];
    __syncthreads();
    const double d = piv;
    if (!(d > 0.0)) {
      bad = true;
      break;
    }
    const double sd = sqrt(d);
    const double lij = i > j ? row[j] / sd : (i == j ? sd : 0.0);
    row[j] = lij;
    colj[i] = lij;
    __syncthreads();
#pragma unroll
    for (int c = j + 1; c < kT; ++c) {  // rows below j, columns up to the diagonal
      const double f = i >= c ? lij : 0.0;
      row[c] = fma(-f, colj[c], row[c]);
    }
    __syncthreads();
  }
  if (bad) {
    if (i == 0) *flag = 1;
    return;
  }
#pragma unroll
  for (int c = 0; c < kT; ++c) Ls[i][c] = c <= i ? row[c] : 0.0;
  __syncthreads();
  for (int r = 0; r < kT; ++r) blk[(size_t)r * N + i] = Ls[r][i];
  // column c = i of Y: y[k] = (delta_kc - sum_{m < k} L[k][m] y[m]) / L[k][k]
  double y[kT];
#pragma unroll
  for (int k = 0; k < kT; ++k) {
    double s = k == i ? 1.0 : 0.0;
#pragma unroll
    for (int m = 0; m < k; ++m) s -= Ls[k][m] * y[m];
    y[k] = k >= i ? s / Ls[k][k] : 0.0;
  }
  double *yo = Yd + (size_t)kb * kT * kT;
#pragma unroll
  for (int k = 0; k < kT; ++k) yo[(size_t)k * kT + i] = y[k];
}

// Panel: L_ik = A_ik L_kk^{-T} for the block rows i > kb (one per workgroup).
__global__ __launch_bounds__(256) void panel_kernel(double *__restrict__ A, int N, int kb,
                                                    const double *__restrict__ Yd) {
  const int i = kb + 1 + blockIdx.x, m0 = (threadIdx.x >> 6) * 16;
  double *tile = A + (size_t)i * kT * N + (size_t)kb * kT;
  const double *y = Yd + (size_t)kb * kT * kT;
  f64x4 acc[4] = {};
  // A(r, k) = tile[r N + k]; B(k, c) = Y[c][k]
  mma16x64<kT>(tile + (size_t)m0 * N, N, 1, y, 1, kT, 0, kT, acc);
  __syncthreads();  // every wavefront has read the tile
  store16x64(tile, N, acc, 0);
}

// Trailing update by nk panels (block columns kb .. kb + nk - 1, K = 64 nk):
// A_ij -= L_i,[kb..] L_j,[kb..]^T over the lower triangle i >= j >= kb + nk;
// with col_only, the tiles (i, kb + 1) for i > kb instead (nk = 1).
__global__ __launch_bounds__(256) void update_kernel(double *__restrict__ A, int N, int kb, int nk,
                                                     int col_only) {
  int i, j;
  if (col_only) {
    i = kb + 1 + (int)blockIdx.x;
    j = kb + 1;
  } else {
    const long long p = blockIdx.x;
    int ii = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((long long)(ii + 1) * (ii + 2) / 2 <= p) ++ii;
    while ((long long)ii * (ii + 1) / 2 > p) --ii;
    const int jj = (int)(p - (long long)ii * (ii + 1) / 2);
    i = kb + nk + ii;
    j = kb + nk + jj;
  }
  const int m0 = (threadIdx.x >> 6) * 16;
  const double *Li = A + (size_t)i * kT * N + (size_t)kb * kT;
  const double *Lj = A + (size_t)j * kT * N + (size_t)kb * kT;
  f64x4 acc[4] = {};
  for (int q = 0; q < nk; ++q)
    mma16x64<kT>(Li + (size_t)m0 * N + q * kT, N, 1, Lj + q * kT, 1, N, 0, kT, acc);
  store16x64(A + (size_t)i * kT * N + (size_t)j * kT, N, acc, 1);
}

__global__ void identity_kernel(double *__restrict__ W, int N) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < N; r += gridDim.x * blockDim.x)
    W[(size_t)r * N + r] = 1.0;
}

// W_i,c = L_ii^{-1} W_i,c for the tiles c <= i of block row i.
__global__ __launch_bounds__(256) void trsm_scale_kernel(double *__restrict__ W, int N, int i,
                                                         const double *__restrict__ Yd) {
  const int c = blockIdx.x, m0 = (threadIdx.x >> 6) * 16;
  double *tile = W + (size_t)i * kT * N + (size_t)c * kT;
  const double *y = Yd + (size_t)i * kT * kT;
  f64x4 acc[4] = {};
  // A(r, k) = Y[r][k]; B(k, c) = tile[k N + c]
  mma16x64<kT>(y + (size_t)m0 * kT, kT, 1, tile, N, 1, 0, kT, acc);
  __syncthreads();  // every wavefront has read the tile
  store16x64(tile, N, acc, 0);
}

// By nk block rows (i .. i + nk - 1, K = 64 nk): W_j,c -= L_j,[i..] W_[i..],c
// for j >= i + nk, c < i + nk (the grid's first (i + nk) tiles are row i + nk).
__global__ __launch_bounds__(256) void trsm_update_kernel(const double *__restrict__ L,
                                                          double *__restrict__ W, int N,
                                                          int i, int nk) {
  const int j = i + nk + blockIdx.x / (i + nk), c = blockIdx.x % (i + nk);
  const int m0 = (threadIdx.x >> 6) * 16;
  const double *Lji = L + (size_t)j * kT * N + (size_t)i * kT;
  const double *Wic = W + (size_t)i * kT * N + (size_t)c * kT;
  f64x4 acc[4] = {};
  for (int q = 0; q < nk; ++q)
    mma16x64<kT>(Lji + (size_t)m0 * N + q * kT, N, 1, Wic + (size_t)q * kT * N, N, 1, 0, kT,
                 acc);
  store16x64(W + (size_t)j * kT * N + (size_t)c * kT, N, acc, 1);
}

// X_ab = sum over block rows k >= a of W_ka^T W_kb for the lower block
// triangle a >= b (X is symmetric).
__global__ __launch_bounds__(256) void xprod_kernel(const double *__restrict__ W, int N,
                                                    double *__restrict__ X) {
  const long long p = blockIdx.x;
  int a = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while ((long long)(a + 1) * (a + 2) / 2 <= p) ++a;
  while ((long long)a * (a + 1) / 2 > p) --a;
  const int bcol = (int)(p - (long long)a * (a + 1) / 2), m0 = (threadIdx.x >> 6) * 16;
  const int k0 = a * kT;
  f64x4 acc[4] = {};
  // A(r, k) = W[k][a 64 + r]; B(k, c) = W[k][b 64 + c]
  mma16x64<0>(W + (size_t)a * kT + m0, 1, N, W + (size_t)bcol * kT, N, 1, k0, N, acc);
  store16x64(X + (size_t)a * kT * N + (size_t)bcol * kT, N, acc, 0);
}

// Upper block triangle of X from the lower one, through a 32 x 32 LDS tile:
// X[r][c] = X[c][r] for the blocks a < b.
__global__ __launch_bounds__(256) void mirror_kernel(double *__restrict__ X, int N) {
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // source tile rows by.., cols bx..
  if ((by / kT) <= (bx / kT)) return;  // source must lie in a strictly lower block
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) t[r][tx] = X[(size_t)(by + r) * N + bx + tx];
  __syncthreads();
  for (int r = ty; r < 32; r += 8) X[(size_t)(bx + r) * N + by + tx] = t[tx][r];
}

// H[l][bus] = b_l (X[f'][bus'] - X[t'][bus']), zero at the slack.
__global__ void gather_kernel(const double *__restrict__ X, int N, const int *__restrict__ fbus,
                              const int *__restrict__ tbus, const double *__restrict__ b,
                              int n_bus, int n_line, int slack, double *__restrict__ H) {
  for (int l = blockIdx.y; l < n_line; l += gridDim.y) {
    const int f = reduced(fbus[l], slack), t = reduced(tbus[l], slack);
    const double bl = b[l];
    for (int bus = blockIdx.x * blockDim.x + threadIdx.x; bus < n_bus;
         bus += gridDim.x * blockDim.x) {
      const int c = reduced(bus, slack);
      double v = 0.0;
      if (c >= 0) {
        const double xf = f >= 0 ? X[(size_t)f * N + c] : 0.0;
        const double xt = t >= 0 ? X[(size_t)t * N + c] : 0.0;
        v = bl * (xf - xt);
      }
      H[(size_t)l * n_bus + bus] = v;
    }
  }
}


__global__ void zero_kernel(double *__restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void zero_flag_kernel(int *flag) { *flag = 0; }

// Device buffers of one build: the two N x N matrices, the inverses of the
// diagonal blocks, the line data, the incidence lists and the failure flag.
struct Workspace {
  double *A = nullptr, *W = nullptr, *Yd = nullptr, *b = nullptr;
  int *start = nullptr, *adj = nullptr, *fbus = nullptr, *tbus = nullptr, *flag = nullptr;
};

dcopf_status validate(int32_t n_bus, int32_t n_line, const int32_t *fbus, const int32_t *tbus,
                      const double *b, int32_t slack, const double *H) {
  if (!fbus || !tbus || !b || !H) return set_error("ptdf: null pointer"), DCOPF_E_INVALID;
  if (n_bus < 2 || n_line < 1) return set_error("ptdf: need n_bus >= 2, n_line >= 1"), DCOPF_E_INVALID;
  if (slack < 0 || slack >= n_bus) return set_error("ptdf: slack out of range"), DCOPF_E_INVALID;
  for (int l = 0; l < n_line; ++l) {
    if (fbus[l] < 0 || fbus[l] >= n_bus || tbus[l] < 0 || tbus[l] >= n_bus)
      return set_error("ptdf: bus index out of range"), DCOPF_E_INVALID;
    if (fbus[l] == tbus[l]) return set_error("ptdf: a line joins a bus to itself"), DCOPF_E_INVALID;
    if (!(std::isfinite(b[l]) && b[l] > 0.0))
      return set_error("ptdf: susceptances must be finite and positive"), DCOPF_E_INVALID;
  }
  return DCOPF_OK;
}

// The build itself, on buffers the caller of this function provides (every
// buffer is cleared or written here before it is read).
dcopf_status build(int32_t n_bus, int32_t n_line, const int32_t *fbus, const int32_t *tbus,
                   const double *b, int32_t slack, hipStream_t s, double *H,
                   const Workspace &ws) {
  const int n = n_bus - 1, T = (n + kT - 1) / kT, N = T * kT;
  // incidence lists per bus, in line order
  std::vector<int> start(n_bus + 1, 0), adj(2 * (size_t)n_line);
  for (int l = 0; l < n_line; ++l) {
    ++start[fbus[l] + 1];
    ++start[tbus[l] + 1];
  }
  for (int i = 0; i < n_bus; ++i) start[i + 1] += start[i];
  {
    std::vector<int> fill(start.begin(), start.end() - 1);
    for (int l = 0; l < n_line; ++l) {
      adj[fill[fbus[l]]++] = l;
      adj[fill[tbus[l]]++] = l;
    }
  }
  const size_t NN = (size_t)N * N;
  double *A = ws.A, *W = ws.W, *Yd = ws.Yd;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
  };
  chk(hipMemcpyAsync(ws.b, b, (size_t)n_line * 8, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(ws.start, start.data(), (size_t)(n_bus + 1) * 4, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(ws.adj, adj.data(), 2 * (size_t)n_line * 4, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(ws.fbus, fbus, (size_t)n_line * 4, hipMemcpyHostToDevice, s));
  chk(hipMemcpyAsync(ws.tbus, tbus, (size_t)n_line * 4, hipMemcpyHostToDevice, s));
  const int gz = (int)std::min<size_t>(4096, (NN + 255) / 256);
  zero_flag_kernel<<<1, 1, 0, s>>>(ws.flag);
  zero_kernel<<<gz, 256, 0, s>>>(A, NN);
  const int g = std::min(1024, (N + 255) / 256);
  assemble_kernel<<<g, 256, 0, s>>>(ws.start, ws.adj, ws.fbus, ws.tbus, ws.b, slack, n, N, A);
  // block columns in pairs: the second column takes the first panel's
  // update alone, then one K = 128 update of the trailing triangle
  for (int kb = 0; kb < T; kb += 2) {
    potrf_kernel<<<1, 64, 0, s>>>(A, N, kb, Yd, ws.flag);
    const int R = T - kb - 1;
    if (R == 0) break;
    panel_kernel<<<R, 256, 0, s>>>(A, N, kb, Yd);
    update_kernel<<<R, 256, 0, s>>>(A, N, kb, 1, 1);
    potrf_kernel<<<1, 64, 0, s>>>(A, N, kb + 1, Yd, ws.flag);
    const int R2 = R - 1;
    if (R2 > 0) {
      panel_kernel<<<R2, 256, 0, s>>>(A, N, kb + 1, Yd);
      update_kernel<<<(unsigned)((long long)R2 * (R2 + 1) / 2), 256, 0, s>>>(A, N, kb, 2, 0);
    }
  }
  zero_kernel<<<gz, 256, 0, s>>>(W, NN);
  identity_kernel<<<g, 256, 0, s>>>(W, N);
  // block rows in pairs: row i + 1 takes row i's update alone, then one
  // K = 128 update of the rows below
  for (int i = 0; i < T; i += 2) {
    trsm_scale_kernel<<<i + 1, 256, 0, s>>>(W, N, i, Yd);
    if (i + 1 == T) break;
    trsm_update_kernel<<<i + 1, 256, 0, s>>>(A, W, N, i, 1);
    trsm_scale_kernel<<<i + 2, 256, 0, s>>>(W, N, i + 1, Yd);
    const int R = T - i - 2;
    if (R > 0)
      trsm_update_kernel<<<(unsigned)((long long)R * (i + 2)), 256, 0, s>>>(A, W, N, i, 2);
  }
  xprod_kernel<<<(unsigned)((long long)T * (T + 1) / 2), 256, 0, s>>>(W, N, A);
  mirror_kernel<<<dim3((unsigned)(N / 32), (unsigned)(N / 32)), 256, 0, s>>>(A, N);
  dim3 gg((unsigned)std::min(64, (n_bus + 255) / 256), (unsigned)std::min(n_line, 32768));
  gather_kernel<<<gg, 256, 0, s>>>(A, N, ws.fbus, ws.tbus, ws.b, n_bus, n_line, slack, H);
  chk(hipGetLastError());
  chk(hipStreamSynchronize(s));
  int hflag = 0;
  if (e == hipSuccess) chk(hipMemcpy(&hflag, ws.flag, 4, hipMemcpyDeviceToHost));
  if (e != hipSuccess) return set_error(std::string("ptdf: ") + hipGetErrorString(e)), DCOPF_E_HIP;
  if (hflag) return set_error("ptdf: the network is not connected"), DCOPF_E_INVALID;
  return DCOPF_OK;
}

// ---------------------------------------------------------------------------
// Fixed workspace of dcopf_ptdf_noalloc: networks of at most
// DCOPF_PTDF_NOALLOC_MAX_BUS buses (N = 2048 reduced rows) and
// DCOPF_PTDF_NOALLOC_MAX_LINE lines.  Each device holds its own copy for the
// life of the process; host code addresses it only through the pointer that
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocN = 2048;
constexpr size_t kOffA = 0;
constexpr size_t kOffW = kOffA + kNoAllocN * kNoAllocN * 8;
constexpr size_t kOffY = kOffW + kNoAllocN * kNoAllocN * 8;
constexpr size_t kOffB = kOffY + kNoAllocN * kT * 8;
constexpr size_t kOffStart = kOffB + (size_t)DCOPF_PTDF_NOALLOC_MAX_LINE * 8;
constexpr size_t kOffAdj = kOffStart + round_up_c((size_t)DCOPF_PTDF_NOALLOC_MAX_BUS + 1, 64) * 4;
constexpr size_t kOffF = kOffAdj + 2 * (size_t)DCOPF_PTDF_NOALLOC_MAX_LINE * 4;
constexpr size_t kOffT = kOffF + (size_t)DCOPF_PTDF_NOALLOC_MAX_LINE * 4;
constexpr size_t kOffFlag = kOffT + (size_t)DCOPF_PTDF_NOALLOC_MAX_LINE * 4;
constexpr size_t kScratchBytes = kOffFlag + 256;
static_assert(kOffStart % 256 == 0 && kOffAdj % 256 == 0 && kOffF % 256 == 0 &&
                  kOffT % 256 == 0 && kOffFlag % 256 == 0,
              "workspace regions stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per
// device, with that device current).
dcopf_status scratch_on_current_device(unsigned char **out) {
  int dev = -1;
  DCOPF_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error("ptdf_noalloc: device index out of range"), DCOPF_E_INVALID;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(std::string("ptdf_noalloc: hipGetSymbolAddress failed: ") +
                       hipGetErrorString(e)),
             DCOPF_E_HIP;
    g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
  }
  *out = g_scratch_ptr[dev];
  return DCOPF_OK;
}

}  // namespace
}  // namespace dcopf

using namespace dcopf;

extern "C" dcopf_status dcopf_ptdf(int32_t n_bus, int32_t n_line, const int32_t *fbus,
                                   const int32_t *tbus, const double *b, int32_t slack,
                                   void *hip_stream, double *H) {
  set_error("");
  dcopf_status st = validate(n_bus, n_line, fbus, tbus, b, slack, H);
  if (st != DCOPF_OK) return st;
  const int n = n_bus - 1, T = (n + kT - 1) / kT, N = T * kT;
  const size_t NN = (size_t)N * N;
  Workspace ws;
  const DevMem mem = current_devmem(hip_stream);
  std::vector<std::pair<void *, size_t>> got;
  auto alloc = [&](void **p, size_t bytes) {
    if (st != DCOPF_OK) return;
    *p = mem.get(bytes);
    if (*p) got.emplace_back(*p, bytes);
    else st = DCOPF_E_NOMEM;
  };
  alloc((void **)&ws.A, NN * 8);
  alloc((void **)&ws.W, NN * 8);
  alloc((void **)&ws.Yd, (size_t)T * kT * kT * 8);
  alloc((void **)&ws.b, (size_t)n_line * 8);
  alloc((void **)&ws.start, (size_t)(n_bus + 1) * 4);
  alloc((void **)&ws.adj, 2 * (size_t)n_line * 4);
  alloc((void **)&ws.fbus, (size_t)n_line * 4);
  alloc((void **)&ws.tbus, (size_t)n_line * 4);
  alloc((void **)&ws.flag, 4);
  if (st == DCOPF_OK) st = build(n_bus, n_line, fbus, tbus, b, slack, (hipStream_t)hip_stream, H, ws);
  else set_error("ptdf: device allocation failed");
  for (auto &g : got) mem.put(g.first, g.second);
  return st;
}

extern "C" dcopf_status dcopf_ptdf_noalloc(int32_t n_bus, int32_t n_line, const int32_t *fbus,
                                           const int32_t *tbus, const double *b, int32_t slack,
                                           void *hip_stream, double *H) {
  set_error("");
  dcopf_status st = validate(n_bus, n_line, fbus, tbus, b, slack, H);
  if (st != DCOPF_OK) return st;
  if (n_bus > DCOPF_PTDF_NOALLOC_MAX_BUS || n_line > DCOPF_PTDF_NOALLOC_MAX_LINE)
    return set_error("ptdf_noalloc: at most " + std::to_string(DCOPF_PTDF_NOALLOC_MAX_BUS) +
                     " buses and " + std::to_string(DCOPF_PTDF_NOALLOC_MAX_LINE) +
                     " lines (fixed workspace); use dcopf_ptdf for larger networks"),
           DCOPF_E_INVALID;
  unsigned char *base = nullptr;
  st = scratch_on_current_device(&base);
  if (st != DCOPF_OK) return st;
  Workspace ws;
  ws.A = reinterpret_cast<double *>(base + kOffA);
  ws.W = reinterpret_cast<double *>(base + kOffW);
  ws.Yd = reinterpret_cast<double *>(base + kOffY);
  ws.b = reinterpret_cast<double *>(base + kOffB);
  ws.start = reinterpret_cast<int *>(base + kOffStart);
  ws.adj = reinterpret_cast<int *>(base + kOffAdj);
  ws.fbus = reinterpret_cast<int *>(base + kOffF);
  ws.tbus = reinterpret_cast<int *>(base + kOffT);
  ws.flag = reinterpret_cast<int *>(base + kOffFlag);
  return build(n_bus, n_line, fbus, tbus, b, slack, (hipStream_t)hip_stream, H, ws);
}
