// Shared device/host helpers of the HIP path (not used by the oracle).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <tuple>
#include <utility>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/dcopf_dual.h"

namespace dcopf {

constexpr int kWave = 64;

// Thread-local last-error message, returned by dcopf_last_error().
void set_error(const std::string &msg);
const char *get_error();

// Device memory of one handle: the caller's allocator (dcopf_set_allocator)
// captured at create, or hipMalloc / hipFree.
struct DevMem {
  dcopf_alloc_fn fa = nullptr;
  dcopf_free_fn ff = nullptr;
  void *ctx = nullptr;
  void *stream = nullptr;
  void *get(size_t bytes) const {
    void *p = nullptr;
    if (!fa) return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
    return fa(bytes, stream, ctx);
  }
  void put(void *p, size_t bytes) const {
    if (!p) return;
    if (!ff) (void)hipFree(p);
    else ff(p, bytes, stream, ctx);
  }
};

// The calling thread's allocator, for work on `stream`.
DevMem current_devmem(void *stream);

// Every buffer a handle owns, returned together at destroy; temporaries are
// returned one by one (put).
struct DevPool {
  DevMem mem;
  std::vector<std::pair<void *, size_t>> bufs;
  void *get(size_t bytes) {
    if (bytes == 0) bytes = 1;
    void *p = mem.get(bytes);
    if (p) bufs.emplace_back(p, bytes);
    return p;
  }
  template <typename T> T *get_n(size_t n) { return static_cast<T *>(get(n * sizeof(T))); }
  void put(void *p) {
    if (!p) return;
    for (size_t i = bufs.size(); i-- > 0;)
      if (bufs[i].first == p) {
        mem.put(p, bufs[i].second);
        bufs.erase(bufs.begin() + (long)i);
        return;
      }
  }
  void release_all() {
    for (size_t i = bufs.size(); i-- > 0;) mem.put(bufs[i].first, bufs[i].second);
    bufs.clear();
  }
};

#define DCOPF_HIP_TRY(expr)                                                    \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::dcopf::set_error(std::string(#expr " failed: ") + hipGetErrorString(e_)); \
      return DCOPF_E_HIP;                                                      \
    }                                                                          \
  } while (0)

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// 16-byte vector of T for coalesced row streaming (clang ext vectors, so the
// nontemporal load builtin accepts them).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> {
  using type = f32x4;
  static constexpr int n = 4;
};
template <> struct Vec16<double> {
  using type = f64x2;
  static constexpr int n = 2;
};

__device__ __forceinline__ float fma_vec(const f32x4 &a, const f32x4 &b, float acc) {
  acc = fmaf(a.x, b.x, acc);
  acc = fmaf(a.y, b.y, acc);
  acc = fmaf(a.z, b.z, acc);
  acc = fmaf(a.w, b.w, acc);
  return acc;
}
__device__ __forceinline__ double fma_vec(const f64x2 &a, const f64x2 &b, double acc) {
  acc = fma(a.x, b.x, acc);
  acc = fma(a.y, b.y, acc);
  return acc;
}

// Sum over the 64 lanes of a wavefront (butterfly; every lane gets the sum,
// the order is fixed so the result is deterministic).
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide deterministic sum of one value per thread (blockDim.x <= 1024,
// multiple of 64).  `scratch` needs blockDim.x / 64 entries.  Every thread
// gets the result.
template <typename T> __device__ __forceinline__ T block_sum(T v, T *scratch) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += scratch[i];
  __syncthreads();
  return s;
}

// Block-wide deterministic sums of NV values per thread in one pass (three
// barriers for all of them); every thread gets the sums.  `scratch` holds
// NV * (blockDim.x / 64) doubles.
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double *scratch) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int c = 0; c < NV; ++c) v[c] = wave_sum(v[c]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < NV; ++c) scratch[c * nw + wave] = v[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += scratch[c * nw + w];
    v[c] = t;
  }
  __syncthreads();
}

// load through a global-address-space pointer (global_load rather than
// flat_load: only the vector memory counter is involved in its waits)
template <typename T> __device__ __forceinline__ T ldg(const T *p) {
  return *(const __attribute__((address_space(1))) T *)(p);
}

// Agent-scope loads/stores for values exchanged between workgroups of one
// launch (cross-XCD visibility).
template <typename T> __device__ __forceinline__ void store_agent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ T load_agent(const T *p) {
  return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// "Last workgroup done" election: every workgroup calls this after storing its
// partial results; exactly one (the last to arrive) gets true and then sees
// every other workgroup's partials.  The counter is reset for the next launch.
__device__ __forceinline__ bool last_block_done(unsigned *counter, bool *flag_smem) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // publish partials
    unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
    bool last = (prev == gridDim.x - 1);
    if (last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *flag_smem = last;
  }
  __syncthreads();
  bool last = *flag_smem;
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}

// Launch `kernel` with the arguments converted to its parameter types.  With
// events e0 != nullptr the start and stop events are attached to the dispatch
// itself (the kernel's own start/end timestamps, as a profiler records them);
// otherwise an ordinary launch (capturable into a HIP graph).
template <typename... KA, typename... A>
inline hipError_t launch_k(void (*kernel)(KA...), dim3 grid, dim3 block, unsigned lds,
                           hipStream_t stream, hipEvent_t e0, hipEvent_t e1, A... args) {
  std::tuple<KA...> t{static_cast<KA>(args)...};
  void *ptrs[sizeof...(KA) > 0 ? sizeof...(KA) : 1];
  std::apply([&](auto &...x) {
    int i = 0;
    ((ptrs[i++] = (void *)&x), ...);
  }, t);
  if (e0)
    return hipExtLaunchKernel((const void *)kernel, grid, block, ptrs, lds, stream, e0, e1, 0);
  return hipLaunchKernel((const void *)kernel, grid, block, ptrs, lds, stream);
}

// ---------------------------------------------------------------------------
// Working-set solve of one repair step, block-wide (every thread of the
// workgroup calls it with the same arguments).  G: Gram matrix of the active
// line rows 0..m-1 and the balance row m (lower triangle, row stride LD,
// left intact); t: targets; sg: directions (+1 / -1) of rows 0..m-1; L:
// factor workspace (LD x LD); y: the multipliers over rows 0..m, zero
// outside the working set.  The active lines are inequalities: starting
// from all of them, a working line whose multiplier pushes its flow out
// (largest sg y > 0) leaves, else the line outside that the step would push
// furthest past its target by more than margin / 2 ((G y)_r - t_r) joins
// again, else the set is final; ties to the lowest row, at most
// 4 (m + 1) + 8 solves, each a Cholesky factorisation (ridge of ridge times
// the largest diagonal) and two triangular solves.  Returns false when a
// pivot was not positive.
//
// The factorisation is right-looking in blocks of kWsNb columns: a block's
// panel (its columns, rows k0 .. n-1) is factored in LDS column by column,
// with the forward substitution riding along, then the
// trailing lower triangle in global memory takes the block's kWsNb updates
// in column order.  The back substitution runs in blocks of kWsNb rows from
// the bottom (a block's rows of L in LDS, its triangle by one wavefront, the
// rows above updated in descending column order).  Every element of the
// factor and of the solution sees the same operations in the same order as
// in the unblocked algorithm, so the result is the same to the last bit;
// what changes is that a column step works on the panel in LDS instead of
// passing over the whole trailing matrix in global memory.
// ---------------------------------------------------------------------------
constexpr int kWsNb = 16;
constexpr int kWsPan = kWsNb + 1;  // row stride (doubles) of the panel in LDS
constexpr int kWsRow = 257;        // row stride (doubles) of a row block in LDS
struct WsShared {
  int wm[256];      // working mask of rows 0..m-1
  int sidx[256];    // working rows in order, then the balance row
  double v[256];    // right-hand side (reduced in place), then the solution, then the join test
  double z[256];    // forward, then back substitution
  double col[256];  // the factor's current column (scaled)
  double red[16];
  // the factor's panel [256][kWsPan] while factoring, its row block
  // [kWsNb][kWsRow] during the back substitution
  double buf[256 * kWsPan > kWsNb * kWsRow ? 256 * kWsPan : kWsNb * kWsRow];
  int ns, pick;
};

template <int LD>
__device__ bool ws_solve(const double *G, const double *t, const int *sg, int m, double *L,
                         double *y, double margin, double ridge, WsShared &sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  auto gl = [&](int a, int b) -> double {
    return a >= b ? G[(size_t)a * LD + b] : G[(size_t)b * LD + a];
  };
  auto l = [&](int a, int b) -> double & { return L[(size_t)a * LD + b]; };
  for (int r = tid; r < m; r += nt) sh.wm[r] = 1;
  __syncthreads();
  const int cap = 4 * (m + 1) + 8;
  for (int pass = 0; pass < cap; ++pass) {
    if (tid == 0) {
      int ns = 0;
      for (int r = 0; r < m; ++r)
        if (sh.wm[r]) sh.sidx[ns++] = r;
      sh.sidx[ns++] = m;
      sh.ns = ns;
    }
    __syncthreads();
    const int n = sh.ns;
    double dm = 0.0;
    for (int a = tid; a < n; a += nt) dm = fmax(dm, gl(sh.sidx[a], sh.sidx[a]));
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) dm = fmax(dm, __shfl_xor(dm, off, kWave));
    if (tid % kWave == 0) sh.red[tid / kWave] = dm;
    __syncthreads();
    dm = 0.0;
    for (int w = 0; w < nt / kWave; ++w) dm = fmax(dm, sh.red[w]);
    if (!(dm > 0.0)) return false;
    // rows of the factor by thread row ty, columns by thread column tx
    const int tx = tid & 31, ty = tid >> 5, ny = nt >> 5;
    for (int a = ty; a < n; a += ny)
      for (int b = tx; b <= a; b += 32)
        l(a, b) = gl(sh.sidx[a], sh.sidx[b]) + (a == b ? ridge * dm : 0.0);
    for (int a = tid; a < n; a += nt) sh.v[a] = t[sh.sidx[a]];
    __syncthreads();
    // blocked right-looking Cholesky with the forward substitution L z = v
    double *pan = sh.buf;
    for (int k0 = 0; k0 < n; k0 += kWsNb) {
      const int kw = min(kWsNb, n - k0), pr = n - k0;
      for (int e = tid; e < pr * kw; e += nt) {
        const int a = k0 + e / kw, c = e % kw;
        pan[(a - k0) * kWsPan + c] = (k0 + c <= a) ? l(a, k0 + c) : 0.0;
      }
      __syncthreads();
      for (int c = 0; c < kw; ++c) {
        const int k = k0 + c;
        const double d = pan[c * kWsPan + c];
        if (!(d > 0.0)) return false;  // the same value in every thread
        const double dk = sqrt(d);
        for (int a = k + 1 + tid; a < n; a += nt) {
          const double q = pan[(a - k0) * kWsPan + c] / dk;
          pan[(a - k0) * kWsPan + c] = q;
          sh.col[a] = q;
        }
        __syncthreads();
        // every thread has read the pivot and the right-hand side's row k
        const double zk = sh.v[k] / dk;
        if (tid == 0) {
          pan[c * kWsPan + c] = dk;
          sh.z[k] = zk;
        }
        for (int a = k + 1 + tid; a < n; a += nt) sh.v[a] -= sh.col[a] * zk;
        // the panel's later columns b (k < b < k0 + kw), rows a >= b
        const int cr = kw - 1 - c;  // columns left in the panel
        for (int e = tid; e < (n - k - 1) * cr; e += nt) {
          const int a = k + 1 + e / cr, b = k + 1 + e % cr;
          if (b <= a) pan[(a - k0) * kWsPan + (b - k0)] -= sh.col[a] * sh.col[b];
        }
        __syncthreads();
      }
      for (int e = tid; e < pr * kw; e += nt) {
        const int a = k0 + e / kw, c = e % kw;
        if (k0 + c <= a) l(a, k0 + c) = pan[(a - k0) * kWsPan + c];
      }
      // trailing lower triangle: the block's columns in order
      const int t0 = k0 + kw;
      for (int a = t0 + ty; a < n; a += ny)
        for (int b = t0 + tx; b <= a; b += 32) {
          double acc = l(a, b);
          for (int c = 0; c < kw; ++c)
            acc -= pan[(a - k0) * kWsPan + c] * pan[(b - k0) * kWsPan + c];
          l(a, b) = acc;
        }
      __syncthreads();
    }
    // back substitution L^T y = z in row blocks from the bottom
    double *rows = sh.buf;
    for (int k1 = n; k1 > 0; k1 -= kWsNb) {
      const int k0 = max(0, k1 - kWsNb), kw = k1 - k0;
      for (int e = tid; e < kw * k1; e += nt) {
        const int r = e / k1, a = e % k1;
        rows[r * kWsRow + a] = (a <= k0 + r) ? l(k0 + r, a) : 0.0;
      }
      __syncthreads();
      if (tid < kWave) {  // the block's triangle: lane r holds z[k0 + r]
        double zr = tid < kw ? sh.z[k0 + tid] : 0.0;
        for (int k = k1 - 1; k >= k0; --k) {
          const double zk = __shfl(zr, k - k0, kWave) / rows[(k - k0) * kWsRow + k];
          if (tid == k - k0) zr = zk;
          else if (tid < k - k0) zr -= rows[(k - k0) * kWsRow + k0 + tid] * zk;
        }
        if (tid < kw) sh.z[k0 + tid] = zr;
      }
      __syncthreads();
      for (int a = tid; a < k0; a += nt) {
        double acc = sh.z[a];
        for (int k = k1 - 1; k >= k0; --k) acc -= rows[(k - k0) * kWsRow + a] * sh.z[k];
        sh.z[a] = acc;
      }
      __syncthreads();
    }
    for (int a = tid; a < n; a += nt) sh.v[a] = sh.z[a];
    __syncthreads();
    for (int r = tid; r <= m; r += nt) y[r] = 0.0;
    __syncthreads();
    for (int a = tid; a < n; a += nt) y[sh.sidx[a]] = sh.v[a];
    __syncthreads();
    if (tid == 0) {  // a working line held against a slack inequality leaves
      double worst = 0.0;
      int pick = -1;
      for (int a = 0; a + 1 < n; ++a) {
        const double val = sg[sh.sidx[a]] * sh.v[a];
        if (val > worst) {
          worst = val;
          pick = sh.sidx[a];
        }
      }
      sh.pick = pick;
    }
    __syncthreads();
    if (sh.pick >= 0) {
      if (tid == 0) sh.wm[sh.pick] = 0;
      __syncthreads();
      continue;
    }
    for (int r = tid; r < m; r += nt) {  // lines outside: end past the target?
      double val = -1.0;
      if (!sh.wm[r]) {
        double gy = 0.0;
        for (int k = 0; k <= m; ++k) gy += gl(r, k) * y[k];
        val = sg[r] * (gy - t[r]);
      }
      sh.v[r] = val;
    }
    __syncthreads();
    if (tid == 0) {
      double worst = 0.5 * margin;
      int pick = -1;
      for (int r = 0; r < m; ++r)
        if (!sh.wm[r] && sh.v[r] > worst) {
          worst = sh.v[r];
          pick = r;
        }
      sh.pick = pick;
    }
    __syncthreads();
    if (sh.pick >= 0) {
      if (tid == 0) sh.wm[sh.pick] = 1;
      __syncthreads();
      continue;
    }
    break;
  }
  return true;
}

}  // namespace dcopf
