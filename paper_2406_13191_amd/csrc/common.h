// Shared device/host helpers of the HIP path (not used by the oracle).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <tuple>
#include <utility>
#include <cstdio>
#include <string>

namespace dcopf {

constexpr int kWave = 64;

// Thread-local last-error message, returned by dcopf_last_error().
void set_error(const std::string &msg);
const char *get_error();

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

}  // namespace dcopf
