// Device helpers shared by the gfx950 kernels: unit roundoff, binomials,
// wave64 reductions and the per-wave LDS workspace convention.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define BBC_WAVE 64

namespace bbc {

// Unit roundoff of round-to-nearest arithmetic.
template <class T>
struct Eps;
template <>
struct Eps<float> {
  static constexpr float u = 5.9604644775390625e-08f;  // 2^-24
};
template <>
struct Eps<double> {
  static constexpr double u = 1.1102230246251565e-16;  // 2^-53
};

// C(n, k) for n <= 20 (exact in FP32).
__host__ __device__ constexpr int binom_i(int n, int k) {
  int r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (k < 0 || k > n) ? 0 : r;
}

template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, BBC_WAVE));
  return v;
}
template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, BBC_WAVE));
  return v;
}
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, BBC_WAVE);
  return v;
}
__device__ __forceinline__ bool wave_all(bool p) { return __ballot(!p) == 0ull; }
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// One workgroup is one wave in the box kernels, so a workgroup barrier is the
// LDS fence between the dependent steps of a box evaluation.
__device__ __forceinline__ void wave_sync() { __syncthreads(); }

__device__ __forceinline__ float fmin_nan_safe(float a, float b) { return a < b ? a : b; }

}  // namespace bbc
