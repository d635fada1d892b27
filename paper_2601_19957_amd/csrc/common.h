// Internal helpers shared by the gfx950 kernels and the host orchestrator.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <math.h>

#include "../../include/sb.h"

namespace sb {

constexpr double kLog2Pi = 1.8378770664093454835606594728112;
constexpr int kWave = 64;
constexpr int kMaxHist = 8;   // largest L-BFGS memory held in registers
constexpr int kMaxComp = 16;  // largest mixture (responsibilities held per row in registers)
constexpr int kMaxMem = 32;   // largest L-BFGS memory (beyond kMaxHist the history is
                              // streamed from memory in each loop of the recursion)

typedef uint16_t bf16_t;  // raw bit pattern; converted with round-to-nearest-even

__host__ __device__ inline bf16_t f32_to_bf16(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  uint32_t u = v.u;
  if ((u & 0x7f800000u) == 0x7f800000u) {  // inf / nan: keep class
    uint16_t h = (uint16_t)(u >> 16);
    if (u & 0x007fffffu) h |= 0x0040u;
    return h;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(bf16_t h) {
  union { uint32_t u; float f; } v;
  v.u = ((uint32_t)h) << 16;
  return v.f;
}

// ---------------------------------------------------------------- reductions
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Max over the wave; NaN inputs are ignored (fmax semantics).
template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over a block of TPB threads (TPB a multiple of 64); every thread gets
// the total.  `red` is LDS scratch of >= TPB/64 elements per value.  Fixed
// order: waves reduce by butterfly, then wave totals are added in order.
template <int TPB, typename T>
__device__ inline T block_sum(T v, T *red) {
  v = wave_sum(v);
  if constexpr (TPB == 64) {
    return v;
  } else {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    T t = red[0];
#pragma unroll
    for (int i = 1; i < TPB / 64; ++i) t += red[i];
    return t;
  }
}

// Several sums at once (N values), same ordering rule.
template <int TPB, int N, typename T>
__device__ inline void block_sum_n(T (&v)[N], T *red) {
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
  if constexpr (TPB > 64) {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0)
#pragma unroll
      for (int j = 0; j < N; ++j) red[j * (TPB / 64) + w] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T t = red[j * (TPB / 64)];
#pragma unroll
      for (int i = 1; i < TPB / 64; ++i) t += red[j * (TPB / 64) + i];
      v[j] = t;
    }
  }
}

template <int TPB, typename T>
__device__ inline T block_max(T v, T *red) {
  v = wave_max(v);
  if constexpr (TPB == 64) {
    return v;
  } else {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    T t = red[0];
#pragma unroll
    for (int i = 1; i < TPB / 64; ++i) t = fmax(t, red[i]);
    return t;
  }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Bump allocator over a caller-provided workspace.
struct Arena {
  char *base = nullptr;
  size_t cap = 0, off = 0;
  bool measure = false;  // only count bytes
  Arena() = default;
  Arena(void *b, size_t c) : base((char *)b), cap(c), off(0), measure(b == nullptr) {}
  template <typename T>
  T *take(size_t n) {
    size_t o = align_up(off);
    off = o + n * sizeof(T);
    if (measure) return nullptr;
    if (off > cap) return nullptr;
    return (T *)(base + o);
  }
  bool ok() const { return measure || off <= cap; }
};

// thread-local last error
void set_error(const char *fmt, ...);
const char *last_error();

#define SB_HIP(expr)                                                                 \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) {                                                          \
      ::sb::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                      __LINE__);                                                     \
      return SB_E_DEVICE;                                                            \
    }                                                                                \
  } while (0)

#define SB_LAUNCH_CHECK() SB_HIP(hipGetLastError())

}  // namespace sb
