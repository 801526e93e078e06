// Learned warm start: dense network n_in -> h1 -> h2 -> n_out (GELU hidden
// layers) trained and evaluated with BF16 matrix-core products (FP32
// accumulation), FP32 master weights and Adam.
//
// Every product of a training step is one "NT" GEMM C[m][n] = sum_k
// A[m][k] B[n][k] with both operands K-contiguous, so each layer keeps its
// activations in both orientations (the epilogue writes the transposed BF16
// copy that the weight-gradient product needs) and each weight matrix has a
// BF16 copy in both orientations (refreshed by the Adam kernel):
//
//   forward   Z1 = X W1^T + b1, H1 = gelu(Z1); Z2 = H1 W2^T + b2,
//             H2 = gelu(Z2); Y = H2 W3^T + b3
//   loss      dY = 2 (Y - T) / (batch n_out)
//   backward  dW3 = dY^T H2, dZ2 = (dY W3) * gelu'(Z2), dW2 = dZ2^T H1,
//             dZ1 = (dZ2 W2) * gelu'(Z1), dW1 = dZ1^T X, db = column sums
//
// All padded dimensions are multiples of 64; padded rows and columns are
// written as zero so they never contribute to a later product.
#include "common.h"
#include "../../include/dcopf_mlp.h"

#include <cmath>
#include <string>
#include <vector>

typedef __bf16 bf16x8m __attribute__((ext_vector_type(8)));
typedef float f32x16m __attribute__((ext_vector_type(16)));

namespace dcopf {
namespace {

enum { EPI_F32 = 0, EPI_HIDDEN = 1, EPI_OUT = 2, EPI_DHID = 3 };

struct Epi {
  int mode, m_real, n_real;
  const float *bias;    // [n_real]
  float *out32;         // EPI_F32: compact [m_real][n_real]; else padded, ld ldo
  int ldo;
  __bf16 *outb;         // padded BF16 copy, ld ldo
  __bf16 *outt;         // transposed BF16 copy, ld ldt
  int ldt;
  const float *zin;     // EPI_DHID: pre-activation, ld ldo
};

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// C tile of 32 x 32 per workgroup; its four wavefronts split K (wavefront w
// takes the 64-deep K steps w, w + 4, ...), each keeping the loads of its
// next step in flight while it multiplies the current one, and their
// accumulators meet in LDS in wavefront order.  Wavefront 0 runs the
// epilogue.  Small products (a batch of a few hundred rows) thus still
// spread over many workgroups, and long K loops are cut four ways.
__global__ __launch_bounds__(256) void gemm_nt_kernel(const __bf16 *__restrict__ A, int lda,
                                                      const __bf16 *__restrict__ Bt, int ldb,
                                                      int K, int Mp, int Np, Epi e) {
  __shared__ float part[3][16][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
  const int r = lane & 31, koff = (lane >> 5) * 8;
  const __bf16 *a = A + (size_t)(m0 + r) * lda + koff;
  const __bf16 *b = Bt + (size_t)(n0 + r) * ldb + koff;
  f32x16m acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.f;
  const int nsteps = K / 64;
  bf16x8m av[2][4], bv[2][4];
  auto fetch = [&](bf16x8m (&qa)[4], bf16x8m (&qb)[4], int step) {
    const int k = min(step, nsteps - 1) * 64;  // clamped: always in range
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      qa[u] = ldg(reinterpret_cast<const bf16x8m *>(a + k + 16 * u));
      qb[u] = ldg(reinterpret_cast<const bf16x8m *>(b + k + 16 * u));
    }
  };
  int st = wave;
  if (st < nsteps) {
    fetch(av[0], bv[0], st);
    fetch(av[1], bv[1], st + 4);
    for (; st + 4 < nsteps; st += 8) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[0][u], bv[0][u], acc, 0, 0, 0);
      fetch(av[0], bv[0], st + 8);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[1][u], bv[1][u], acc, 0, 0, 0);
      fetch(av[1], bv[1], st + 12);
    }
    if (st < nsteps)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[0][u], bv[0][u], acc, 0, 0, 0);
  }
  if (wave > 0)
#pragma unroll
    for (int j = 0; j < 16; ++j) part[wave - 1][j][lane] = acc[j];
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = ((acc[j] + part[0][j][lane]) + part[1][j][lane]) + part[2][j][lane];
  const int n = n0 + r;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int m = m0 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
    const bool ok = m < e.m_real && n < e.n_real;
    const float v = acc[j];
    if (e.mode == EPI_F32) {
      if (ok) e.out32[(size_t)m * e.n_real + n] = v;
    } else if (e.mode == EPI_HIDDEN) {
      const float z = ok ? v + e.bias[n] : 0.f;
      const float h = ok ? gelu_f(z) : 0.f;
      e.out32[(size_t)m * e.ldo + n] = z;
      e.outb[(size_t)m * e.ldo + n] = (__bf16)h;
      e.outt[(size_t)n * e.ldt + m] = (__bf16)h;
    } else if (e.mode == EPI_OUT) {
      e.out32[(size_t)m * e.ldo + n] = ok ? v + e.bias[n] : 0.f;
    } else {
      const float dz = ok ? v * gelu_grad_f(e.zin[(size_t)m * e.ldo + n]) : 0.f;
      e.out32[(size_t)m * e.ldo + n] = dz;
      e.outb[(size_t)m * e.ldo + n] = (__bf16)dz;
      e.outt[(size_t)n * e.ldt + m] = (__bf16)dz;
    }
  }
}

// X (compact FP32 [batch][n_in]) -> padded BF16 [Bp][I] and its transpose.
__global__ void input_kernel(const float *__restrict__ X, int batch, int n_in, int Mp, int I,
                             int ldt, __bf16 *__restrict__ Xb, __bf16 *__restrict__ Xt) {
  const int m = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < I; i += gridDim.x * blockDim.x) {
    const float v = (m < batch && i < n_in) ? X[(size_t)m * n_in + i] : 0.f;
    const __bf16 b = (__bf16)v;
    Xb[(size_t)m * I + i] = b;
    Xt[(size_t)i * ldt + m] = b;
  }
}

// dY = 2 (Y - T) / (batch n_out) with padding zeroed; per-workgroup partial
// sums of (Y - T)^2 (rows = blockIdx.y).
__global__ __launch_bounds__(256) void loss_kernel(const float *__restrict__ Y, int O,
                                                   const float *__restrict__ T, int batch,
                                                   int n_out, int ldt, float scale,
                                                   float *__restrict__ dY32,
                                                   __bf16 *__restrict__ dYb,
                                                   __bf16 *__restrict__ dYt,
                                                   double *__restrict__ part) {
  __shared__ double red[4];
  const int m = blockIdx.y;
  double s = 0.0;
  for (int o = threadIdx.x; o < O; o += blockDim.x) {
    float d = 0.f;
    if (m < batch && o < n_out) {
      const float rr = Y[(size_t)m * O + o] - T[(size_t)m * n_out + o];
      s += (double)rr * rr;
      d = scale * rr;
    }
    dY32[(size_t)m * O + o] = d;
    dYb[(size_t)m * O + o] = (__bf16)d;
    dYt[(size_t)o * ldt + m] = (__bf16)d;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[m] = s;
}

__global__ __launch_bounds__(256) void loss_sum_kernel(const double *__restrict__ part, int n,
                                                       double inv, double *__restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s * inv;
}

// db[n] = sum over the batch rows of d[m][n] (fixed order).
// Column sums (bias gradients): a workgroup owns 64 columns; its four
// wavefronts each add a quarter of the rows, eight independent rows at a
// time (lane = column, coalesced), and the quarters meet in LDS in order.
__global__ __launch_bounds__(256) void colsum_kernel(const float *__restrict__ d, int ld,
                                                     int batch, int n_real,
                                                     float *__restrict__ db) {
  __shared__ float q[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  const int nc = n < n_real ? n : 0;
  const int per = (batch + 3) / 4, r0 = wave * per, r1 = min(batch, r0 + per);
  float acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.f;
  int m = r0;
  for (; m + 8 <= r1; m += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += d[(size_t)(m + u) * ld + nc];
  for (; m < r1; ++m) acc[0] += d[(size_t)m * ld + nc];
  q[wave][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (wave == 0 && n < n_real) db[n] = ((q[0][lane] + q[1][lane]) + q[2][lane]) + q[3][lane];
}

// Adam on the FP32 masters (compact parameter vector).
__global__ void adam_kernel(float *__restrict__ p, float *__restrict__ mo, float *__restrict__ ve,
                            const float *__restrict__ g, size_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float m = b1 * mo[i] + (1.f - b1) * gi;
    const float v = b2 * ve[i] + (1.f - b2) * gi * gi;
    mo[i] = m;
    ve[i] = v;
    p[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
  }
}

// BF16 copies of W [out][in] (compact FP32): W_b [OUTp][INp], W_t [INp][OUTp].
// BF16 copies of a weight matrix in both orientations, through a 64 x 64
// LDS tile so that both the row-major and the transposed writes are
// coalesced; padded rows and columns are written as zero.
__global__ __launch_bounds__(256) void wcopy_kernel(const float *__restrict__ W, int out, int in,
                                                    int OUTp, int INp, __bf16 *__restrict__ Wb,
                                                    __bf16 *__restrict__ Wt) {
  __shared__ __bf16 t[64][66];
  const int o0 = blockIdx.y * 64, i0 = blockIdx.x * 64;
  const int c = threadIdx.x & 63, r4 = threadIdx.x >> 6;
  for (int r = r4; r < 64; r += 4) {
    const int o = o0 + r, i = i0 + c;
    const float v = (o < out && i < in) ? W[(size_t)o * in + i] : 0.f;
    const __bf16 b = (__bf16)v;
    t[r][c] = b;
    Wb[(size_t)o * INp + i] = b;
  }
  __syncthreads();
  for (int r = r4; r < 64; r += 4) Wt[(size_t)(i0 + r) * OUTp + o0 + c] = t[c][r];
}

// Column mean and standard deviation of A [rows][cols] (FP64 sums; one
// workgroup per 64 columns, its four wavefronts each a quarter of the rows,
// lane = column, quarters combined in order).
__global__ __launch_bounds__(256) void colstats_kernel(const float *__restrict__ A, int rows,
                                                       int cols, float *__restrict__ mean,
                                                       float *__restrict__ sd) {
  __shared__ double q[2][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const int cc = c < cols ? c : 0;
  const int per = (rows + 3) / 4, r0 = wave * per, r1 = min(rows, r0 + per);
  double s = 0.0;
  for (int r = r0; r < r1; ++r) s += (double)A[(size_t)r * cols + cc];
  q[0][wave][lane] = s;
  __syncthreads();
  const double mu = (((q[0][0][lane] + q[0][1][lane]) + q[0][2][lane]) + q[0][3][lane]) / rows;
  double v = 0.0;
  for (int r = r0; r < r1; ++r) {
    const double d = (double)A[(size_t)r * cols + cc] - mu;
    v += d * d;
  }
  q[1][wave][lane] = v;
  __syncthreads();
  if (wave == 0 && c < cols) {
    const double var = (((q[1][0][lane] + q[1][1][lane]) + q[1][2][lane]) + q[1][3][lane]) / rows;
    const double sdv = sqrt(var);
    mean[c] = (float)mu;
    sd[c] = sdv > 1e-12 * (fabs(mu) + 1.0) ? (float)sdv : 1.0f;
  }
}

__global__ void standardize_kernel(const float *__restrict__ A, int rows, int cols,
                                   const float *__restrict__ mean, const float *__restrict__ sd,
                                   int inverse, float *__restrict__ out) {
  const size_t n = (size_t)rows * cols;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % cols);
    out[i] = inverse ? A[i] * sd[c] + mean[c] : (A[i] - mean[c]) / sd[c];
  }
}

// First layer on raw inputs: b1 <- b1 - W1 (mean_x / std_x) (one thread per
// output row, FP64 sum in column order), then W1 <- W1 / std_x.
__global__ void fold_in_kernel(float *__restrict__ W1, float *__restrict__ b1, int out, int in,
                               const float *__restrict__ mx, const float *__restrict__ sx) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= out) return;
  float *w = W1 + (size_t)o * in;
  double t = 0.0;
  for (int i = 0; i < in; ++i) t += (double)w[i] * ((double)mx[i] / (double)sx[i]);
  b1[o] = (float)((double)b1[o] - t);
  for (int i = 0; i < in; ++i) w[i] = (float)((double)w[i] / (double)sx[i]);
}

// Last layer to raw outputs: W3 <- std_y W3 (per row), b3 <- std_y b3 + mean_y.
__global__ void fold_out_kernel(float *__restrict__ W3, float *__restrict__ b3, int out, int in,
                                const float *__restrict__ my, const float *__restrict__ sy) {
  const int o = blockIdx.y;
  const double so = sy[o];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < in; i += gridDim.x * blockDim.x)
    W3[(size_t)o * in + i] = (float)(so * (double)W3[(size_t)o * in + i]);
  if (blockIdx.x == 0 && threadIdx.x == 0) b3[o] = (float)(so * (double)b3[o] + (double)my[o]);
}

// compact Y [batch][n_out] from the padded Y
__global__ void yout_kernel(const float *__restrict__ Yp, int O, int batch, int n_out,
                            float *__restrict__ Y) {
  const int m = blockIdx.y;
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < n_out; o += gridDim.x * blockDim.x)
    Y[(size_t)m * n_out + o] = Yp[(size_t)m * O + o];
}

}  // namespace
}  // namespace dcopf

using namespace dcopf;

struct dcopf_mlp_s {
  dcopf_mlp_config cfg{};
  hipStream_t stream = nullptr;
  int I = 0, A1 = 0, A2 = 0, O = 0, Bm = 0;
  size_t off[7] = {};  // offsets of W1, b1, W2, b2, W3, b3 in the parameter vector; off[6] = total
  float *p = nullptr, *mo = nullptr, *ve = nullptr, *g = nullptr;
  __bf16 *W1b = nullptr, *W1t = nullptr, *W2b = nullptr, *W2t = nullptr, *W3b = nullptr,
         *W3t = nullptr;
  __bf16 *Xb = nullptr, *Xt = nullptr, *H1b = nullptr, *H1t = nullptr, *H2b = nullptr,
         *H2t = nullptr, *dYb = nullptr, *dYt = nullptr, *dZ2b = nullptr, *dZ2t = nullptr,
         *dZ1b = nullptr, *dZ1t = nullptr;
  float *Z1 = nullptr, *Z2 = nullptr, *Y = nullptr, *dY32 = nullptr, *dZ2 = nullptr,
        *dZ1 = nullptr;
  double *part = nullptr, *loss = nullptr;
  long long t = 0;
  DevPool pool;  // every device buffer of the network (the caller's allocator)
};

namespace {

template <typename T> T *malloc_m(dcopf_mlp_s *m, size_t n, bool *ok) {
  T *p = m->pool.get_n<T>(std::max<size_t>(n, 1));
  if (!p) *ok = false;
  return p;
}

void free_mlp(dcopf_mlp_s *m) {
  if (!m) return;
  m->pool.release_all();
  delete m;
}

void gemm(dcopf_mlp_s *m, const __bf16 *A, int lda, const __bf16 *Bt, int ldb, int K, int Mp,
          int Np, const Epi &e) {
  dim3 grid((unsigned)(Np / 32), (unsigned)(Mp / 32));
  gemm_nt_kernel<<<grid, 256, 0, m->stream>>>(A, lda, Bt, ldb, K, Mp, Np, e);
}

void refresh_weights(dcopf_mlp_s *m) {
  const dcopf_mlp_config &c = m->cfg;
  hipStream_t s = m->stream;
  // padded extents are multiples of 64: the 64 x 64 tiles cover them exactly
  wcopy_kernel<<<dim3((unsigned)(m->I / 64), (unsigned)(m->A1 / 64)), 256, 0, s>>>(
      m->p + m->off[0], c.h1, c.n_in, m->A1, m->I, m->W1b, m->W1t);
  wcopy_kernel<<<dim3((unsigned)(m->A1 / 64), (unsigned)(m->A2 / 64)), 256, 0, s>>>(
      m->p + m->off[2], c.h2, c.h1, m->A2, m->A1, m->W2b, m->W2t);
  wcopy_kernel<<<dim3((unsigned)(m->A2 / 64), (unsigned)(m->O / 64)), 256, 0, s>>>(
      m->p + m->off[4], c.n_out, c.h2, m->O, m->A2, m->W3b, m->W3t);
}

void forward_pass(dcopf_mlp_s *m, const float *X, int batch) {
  const dcopf_mlp_config &c = m->cfg;
  hipStream_t s = m->stream;
  const int Mp = (int)round_up(batch, 64);
  input_kernel<<<dim3((unsigned)((m->I + 255) / 256), (unsigned)Mp), 256, 0, s>>>(
      X, batch, c.n_in, Mp, m->I, m->Bm, m->Xb, m->Xt);
  Epi e1{EPI_HIDDEN, batch, c.h1, m->p + m->off[1], m->Z1, m->A1, m->H1b, m->H1t, m->Bm, nullptr};
  gemm(m, m->Xb, m->I, m->W1b, m->I, m->I, Mp, m->A1, e1);
  Epi e2{EPI_HIDDEN, batch, c.h2, m->p + m->off[3], m->Z2, m->A2, m->H2b, m->H2t, m->Bm, nullptr};
  gemm(m, m->H1b, m->A1, m->W2b, m->A1, m->A1, Mp, m->A2, e2);
  Epi e3{EPI_OUT, batch, c.n_out, m->p + m->off[5], m->Y, m->O, nullptr, nullptr, 0, nullptr};
  gemm(m, m->H2b, m->A2, m->W3b, m->A2, m->A2, Mp, m->O, e3);
}

void backward_pass(dcopf_mlp_s *m, const float *T, int batch) {
  const dcopf_mlp_config &c = m->cfg;
  hipStream_t s = m->stream;
  const int Mp = (int)round_up(batch, 64);
  const float scale = 2.0f / ((float)batch * (float)c.n_out);
  loss_kernel<<<dim3(1, (unsigned)Mp), 256, 0, s>>>(m->Y, m->O, T, batch, c.n_out, m->Bm, scale,
                                                    m->dY32, m->dYb, m->dYt, m->part);
  loss_sum_kernel<<<1, 256, 0, s>>>(m->part, Mp, 1.0 / ((double)batch * c.n_out), m->loss);
  // dW3 = dY^T H2 ; db3
  Epi g3{EPI_F32, c.n_out, c.h2, nullptr, m->g + m->off[4], 0, nullptr, nullptr, 0, nullptr};
  gemm(m, m->dYt, m->Bm, m->H2t, m->Bm, Mp, m->O, m->A2, g3);
  colsum_kernel<<<(c.n_out + 63) / 64, 256, 0, s>>>(m->dY32, m->O, batch, c.n_out,
                                                      m->g + m->off[5]);
  // dZ2 = (dY W3) * gelu'(Z2)
  Epi d2{EPI_DHID, batch, c.h2, nullptr, m->dZ2, m->A2, m->dZ2b, m->dZ2t, m->Bm, m->Z2};
  gemm(m, m->dYb, m->O, m->W3t, m->O, m->O, Mp, m->A2, d2);
  Epi g2{EPI_F32, c.h2, c.h1, nullptr, m->g + m->off[2], 0, nullptr, nullptr, 0, nullptr};
  gemm(m, m->dZ2t, m->Bm, m->H1t, m->Bm, Mp, m->A2, m->A1, g2);
  colsum_kernel<<<(c.h2 + 63) / 64, 256, 0, s>>>(m->dZ2, m->A2, batch, c.h2, m->g + m->off[3]);
  // dZ1 = (dZ2 W2) * gelu'(Z1)
  Epi d1{EPI_DHID, batch, c.h1, nullptr, m->dZ1, m->A1, m->dZ1b, m->dZ1t, m->Bm, m->Z1};
  gemm(m, m->dZ2b, m->A2, m->W2t, m->A2, m->A2, Mp, m->A1, d1);
  Epi g1{EPI_F32, c.h1, c.n_in, nullptr, m->g + m->off[0], 0, nullptr, nullptr, 0, nullptr};
  gemm(m, m->dZ1t, m->Bm, m->Xt, m->Bm, Mp, m->A1, m->I, g1);
  colsum_kernel<<<(c.h1 + 63) / 64, 256, 0, s>>>(m->dZ1, m->A1, batch, c.h1, m->g + m->off[1]);
}

void adam(dcopf_mlp_s *m, double lr) {
  m->t += 1;
  const dcopf_mlp_config &c = m->cfg;
  const float c1 = (float)(1.0 - std::pow(c.beta1, (double)m->t));
  const float c2 = (float)(1.0 - std::pow(c.beta2, (double)m->t));
  adam_kernel<<<2048, 256, 0, m->stream>>>(m->p, m->mo, m->ve, m->g, m->off[6], (float)lr,
                                          (float)c.beta1, (float)c.beta2, (float)c.eps, c1, c2);
  refresh_weights(m);
}

dcopf_status check_batch(dcopf_mlp_s *m, const void *X, int batch) {
  if (!m || !X) return set_error("null argument"), DCOPF_E_INVALID;
  if (batch < 1 || batch > m->cfg.max_batch)
    return set_error("batch must be in [1, max_batch]"), DCOPF_E_INVALID;
  return DCOPF_OK;
}

}  // namespace

extern "C" {

dcopf_status dcopf_mlp_create(const dcopf_mlp_config *cfg, void *hip_stream, dcopf_mlp_t *out) {
  if (!out) return set_error("out is NULL"), DCOPF_E_INVALID;
  *out = nullptr;
  if (!cfg) return set_error("null config"), DCOPF_E_INVALID;
  const dcopf_mlp_config &c = *cfg;
  const int dims[4] = {c.n_in, c.h1, c.h2, c.n_out};
  for (int d : dims)
    if (d < 1 || d > 65536) return set_error("layer widths must be in [1, 65536]"), DCOPF_E_INVALID;
  if (c.max_batch < 1 || c.max_batch > 65536)
    return set_error("max_batch must be in [1, 65536]"), DCOPF_E_INVALID;
  if (!(c.beta1 >= 0 && c.beta1 < 1 && c.beta2 >= 0 && c.beta2 < 1 && c.eps > 0))
    return set_error("Adam parameters out of range"), DCOPF_E_INVALID;
  auto *m = new dcopf_mlp_s();
  m->cfg = c;
  m->stream = (hipStream_t)hip_stream;
  m->pool.mem = current_devmem(hip_stream);
  m->I = (int)round_up(c.n_in, 64);
  m->A1 = (int)round_up(c.h1, 64);
  m->A2 = (int)round_up(c.h2, 64);
  m->O = (int)round_up(c.n_out, 64);
  m->Bm = (int)round_up(c.max_batch, 64);
  const size_t sz[6] = {(size_t)c.h1 * c.n_in, (size_t)c.h1, (size_t)c.h2 * c.h1, (size_t)c.h2,
                        (size_t)c.n_out * c.h2, (size_t)c.n_out};
  m->off[0] = 0;
  for (int i = 0; i < 6; ++i) m->off[i + 1] = m->off[i] + sz[i];
  const size_t P = m->off[6];
  const size_t I = m->I, A1 = m->A1, A2 = m->A2, O = m->O, Bm = m->Bm;
  bool ok = true;
  m->p = malloc_m<float>(m, P, &ok);
  m->mo = malloc_m<float>(m, P, &ok);
  m->ve = malloc_m<float>(m, P, &ok);
  m->g = malloc_m<float>(m, P, &ok);
  m->W1b = malloc_m<__bf16>(m, A1 * I, &ok);
  m->W1t = malloc_m<__bf16>(m, I * A1, &ok);
  m->W2b = malloc_m<__bf16>(m, A2 * A1, &ok);
  m->W2t = malloc_m<__bf16>(m, A1 * A2, &ok);
  m->W3b = malloc_m<__bf16>(m, O * A2, &ok);
  m->W3t = malloc_m<__bf16>(m, A2 * O, &ok);
  m->Xb = malloc_m<__bf16>(m, Bm * I, &ok);
  m->Xt = malloc_m<__bf16>(m, I * Bm, &ok);
  m->H1b = malloc_m<__bf16>(m, Bm * A1, &ok);
  m->H1t = malloc_m<__bf16>(m, A1 * Bm, &ok);
  m->H2b = malloc_m<__bf16>(m, Bm * A2, &ok);
  m->H2t = malloc_m<__bf16>(m, A2 * Bm, &ok);
  m->dYb = malloc_m<__bf16>(m, Bm * O, &ok);
  m->dYt = malloc_m<__bf16>(m, O * Bm, &ok);
  m->dZ2b = malloc_m<__bf16>(m, Bm * A2, &ok);
  m->dZ2t = malloc_m<__bf16>(m, A2 * Bm, &ok);
  m->dZ1b = malloc_m<__bf16>(m, Bm * A1, &ok);
  m->dZ1t = malloc_m<__bf16>(m, A1 * Bm, &ok);
  m->Z1 = malloc_m<float>(m, Bm * A1, &ok);
  m->Z2 = malloc_m<float>(m, Bm * A2, &ok);
  m->Y = malloc_m<float>(m, Bm * O, &ok);
  m->dY32 = malloc_m<float>(m, Bm * O, &ok);
  m->dZ2 = malloc_m<float>(m, Bm * A2, &ok);
  m->dZ1 = malloc_m<float>(m, Bm * A1, &ok);
  m->part = malloc_m<double>(m, Bm, &ok);
  m->loss = malloc_m<double>(m, 1, &ok);
  if (!ok) {
    free_mlp(m);
    return set_error("device allocation failed"), DCOPF_E_NOMEM;
  }
  hipError_t e = hipSuccess;
  float *zero[] = {m->p, m->mo, m->ve, m->g};
  for (float *z : zero)
    if (e == hipSuccess) e = hipMemsetAsync(z, 0, P * 4, m->stream);
  // transposed activation buffers: columns beyond a batch stay zero
  __bf16 *tz[] = {m->Xt, m->H1t, m->H2t, m->dYt, m->dZ2t, m->dZ1t};
  const size_t tn[] = {I * Bm, A1 * Bm, A2 * Bm, O * Bm, A2 * Bm, A1 * Bm};
  for (int i = 0; i < 6; ++i)
    if (e == hipSuccess) e = hipMemsetAsync(tz[i], 0, tn[i] * 2, m->stream);
  refresh_weights(m);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    free_mlp(m);
    return set_error(std::string("HIP error in mlp create: ") + hipGetErrorString(e)),
           DCOPF_E_HIP;
  }
  *out = m;
  return DCOPF_OK;
}

size_t dcopf_mlp_param_count(dcopf_mlp_t m) { return m ? m->off[6] : 0; }

dcopf_status dcopf_mlp_get_params(dcopf_mlp_t m, float *params, size_t len) {
  if (!m || !params) return set_error("null argument"), DCOPF_E_INVALID;
  if (len != m->off[6]) return set_error("parameter length mismatch"), DCOPF_E_STATE;
  DCOPF_HIP_TRY(hipStreamSynchronize(m->stream));
  DCOPF_HIP_TRY(hipMemcpy(params, m->p, len * 4, hipMemcpyDeviceToHost));
  return DCOPF_OK;
}

dcopf_status dcopf_mlp_set_params(dcopf_mlp_t m, const float *params, size_t len) {
  if (!m || !params) return set_error("null argument"), DCOPF_E_INVALID;
  if (len != m->off[6]) return set_error("parameter length mismatch"), DCOPF_E_STATE;
  for (size_t i = 0; i < len; ++i)
    if (!std::isfinite(params[i])) return set_error("non-finite parameter"), DCOPF_E_INVALID;
  DCOPF_HIP_TRY(hipStreamSynchronize(m->stream));
  DCOPF_HIP_TRY(hipMemcpy(m->p, params, len * 4, hipMemcpyHostToDevice));
  DCOPF_HIP_TRY(hipMemset(m->mo, 0, len * 4));
  DCOPF_HIP_TRY(hipMemset(m->ve, 0, len * 4));
  m->t = 0;
  refresh_weights(m);
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(m->stream));
  return DCOPF_OK;
}

dcopf_status dcopf_mlp_forward(dcopf_mlp_t m, const float *X, int32_t batch, float *Y) {
  dcopf_status st = check_batch(m, X, batch);
  if (st != DCOPF_OK) return st;
  if (!Y) return set_error("null output"), DCOPF_E_INVALID;
  forward_pass(m, X, batch);
  yout_kernel<<<dim3((unsigned)((m->cfg.n_out + 255) / 256), (unsigned)batch), 256, 0,
                m->stream>>>(m->Y, m->O, batch, m->cfg.n_out, Y);
  DCOPF_HIP_TRY(hipGetLastError());
  return DCOPF_OK;
}

dcopf_status dcopf_mlp_train_step(dcopf_mlp_t m, const float *X, const float *T, int32_t batch,
                                  double lr, double *loss) {
  dcopf_status st = check_batch(m, X, batch);
  if (st != DCOPF_OK) return st;
  if (!T || !(lr > 0) || !std::isfinite(lr)) return set_error("bad targets or lr"), DCOPF_E_INVALID;
  forward_pass(m, X, batch);
  backward_pass(m, T, batch);
  adam(m, lr);
  DCOPF_HIP_TRY(hipGetLastError());
  if (loss) {
    DCOPF_HIP_TRY(hipMemcpyAsync(loss, m->loss, 8, hipMemcpyDeviceToHost, m->stream));
    DCOPF_HIP_TRY(hipStreamSynchronize(m->stream));
    if (!std::isfinite(*loss)) return set_error("non-finite loss"), DCOPF_E_NONFINITE;
  }
  return DCOPF_OK;
}

dcopf_status dcopf_mlp_get_grads(dcopf_mlp_t m, float *grads, size_t len) {
  if (!m || !grads) return set_error("null argument"), DCOPF_E_INVALID;
  if (len != m->off[6]) return set_error("gradient length mismatch"), DCOPF_E_STATE;
  DCOPF_HIP_TRY(hipStreamSynchronize(m->stream));
  DCOPF_HIP_TRY(hipMemcpy(grads, m->g, len * 4, hipMemcpyDeviceToHost));
  return DCOPF_OK;
}

dcopf_status dcopf_mlp_time_train(dcopf_mlp_t m, const float *X, const float *T, int32_t batch,
                                  int32_t n, double *ms) {
  dcopf_status st = check_batch(m, X, batch);
  if (st != DCOPF_OK) return st;
  if (!T || !ms || n < 1) return set_error("bad arguments"), DCOPF_E_INVALID;
  const size_t P = m->off[6];
  std::vector<float> save(P), savem(P), savev(P);
  DCOPF_HIP_TRY(hipStreamSynchronize(m->stream));
  DCOPF_HIP_TRY(hipMemcpy(save.data(), m->p, P * 4, hipMemcpyDeviceToHost));
  DCOPF_HIP_TRY(hipMemcpy(savem.data(), m->mo, P * 4, hipMemcpyDeviceToHost));
  DCOPF_HIP_TRY(hipMemcpy(savev.data(), m->ve, P * 4, hipMemcpyDeviceToHost));
  const long long t0 = m->t;
  hipEvent_t e0, e1;
  DCOPF_HIP_TRY(hipEventCreate(&e0));
  DCOPF_HIP_TRY(hipEventCreate(&e1));
  DCOPF_HIP_TRY(hipEventRecord(e0, m->stream));
  for (int i = 0; i < n; ++i) {
    forward_pass(m, X, batch);
    backward_pass(m, T, batch);
    adam(m, 1e-6);
  }
  DCOPF_HIP_TRY(hipEventRecord(e1, m->stream));
  DCOPF_HIP_TRY(hipEventSynchronize(e1));
  float el = 0.f;
  DCOPF_HIP_TRY(hipEventElapsedTime(&el, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = el / n;
  DCOPF_HIP_TRY(hipMemcpy(m->p, save.data(), P * 4, hipMemcpyHostToDevice));
  DCOPF_HIP_TRY(hipMemcpy(m->mo, savem.data(), P * 4, hipMemcpyHostToDevice));
  DCOPF_HIP_TRY(hipMemcpy(m->ve, savev.data(), P * 4, hipMemcpyHostToDevice));
  m->t = t0;
  refresh_weights(m);
  DCOPF_HIP_TRY(hipGetLastError());
  DCOPF_HIP_TRY(hipStreamSynchronize(m->stream));
  return DCOPF_OK;
}

dcopf_status dcopf_mlp_column_stats(dcopf_mlp_t m, const float *A, int32_t rows, int32_t cols,
                                    float *mean, float *std) {
  if (!m || !A || !mean || !std || rows < 1 || cols < 1)
    return set_error("column_stats: bad arguments"), DCOPF_E_INVALID;
  colstats_kernel<<<(cols + 63) / 64, 256, 0, m->stream>>>(A, rows, cols, mean, std);
  DCOPF_HIP_TRY(hipGetLastError());
  return DCOPF_OK;
}

dcopf_status dcopf_mlp_standardize(dcopf_mlp_t m, const float *A, int32_t rows, int32_t cols,
                                   const float *mean, const float *std, int32_t inverse,
                                   float *out) {
  if (!m || !A || !mean || !std || !out || rows < 1 || cols < 1)
    return set_error("standardize: bad arguments"), DCOPF_E_INVALID;
  const size_t n = (size_t)rows * cols;
  const int g = (int)std::min<size_t>(4096, (n + 255) / 256);
  standardize_kernel<<<g, 256, 0, m->stream>>>(A, rows, cols, mean, std, inverse ? 1 : 0, out);
  DCOPF_HIP_TRY(hipGetLastError());
  return DCOPF_OK;
}

dcopf_status dcopf_mlp_fold_standardizers(dcopf_mlp_t m, const float *x_mean,
                                          const float *x_std, const float *y_mean,
                                          const float *y_std) {
  if (!m || !x_mean || !x_std || !y_mean || !y_std)
    return set_error("fold_standardizers: null pointer"), DCOPF_E_INVALID;
  const dcopf_mlp_config &c = m->cfg;
  hipStream_t s = m->stream;
  fold_in_kernel<<<(c.h1 + 255) / 256, 256, 0, s>>>(m->p + m->off[0], m->p + m->off[1], c.h1,
                                                     c.n_in, x_mean, x_std);
  fold_out_kernel<<<dim3((unsigned)std::min(64, (c.h2 + 255) / 256), (unsigned)c.n_out), 256, 0,
                    s>>>(m->p + m->off[4], m->p + m->off[5], c.n_out, c.h2, y_mean, y_std);
  DCOPF_HIP_TRY(hipMemsetAsync(m->mo, 0, m->off[6] * 4, s));
  DCOPF_HIP_TRY(hipMemsetAsync(m->ve, 0, m->off[6] * 4, s));
  m->t = 0;
  refresh_weights(m);
  DCOPF_HIP_TRY(hipGetLastError());
  return DCOPF_OK;
}

void dcopf_mlp_destroy(dcopf_mlp_t m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  free_mlp(m);
}

}  // extern "C"
