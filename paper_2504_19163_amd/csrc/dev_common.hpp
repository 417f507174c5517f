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

// A workgroup barrier is the LDS fence between the dependent steps of a box
// evaluation (one wave, or NT lanes of several waves, per box).
__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// Reductions over NT threads: a group of NT < 64 lanes of one wave (aligned to
// NT), the wave, or NT a multiple of 64 across the workgroup's waves (through
// LDS).  Every thread of the group must call them.
template <int NT>
__device__ __forceinline__ bool blk_all(bool p) {
  if constexpr (NT == BBC_WAVE) {
    return wave_all(p);
  } else if constexpr (NT < BBC_WAVE) {  // the NT-lane group of this lane
    const uint64_t b = __ballot(!p);
    const int g = int(threadIdx.x % BBC_WAVE) / NT;
    return ((b >> (g * NT)) & ((1ull << NT) - 1ull)) == 0ull;
  } else {
    __shared__ int red[NT / BBC_WAVE];
    const bool w = wave_all(p);
    __syncthreads();
    if ((threadIdx.x % BBC_WAVE) == 0) red[threadIdx.x / BBC_WAVE] = w ? 1 : 0;
    __syncthreads();
    bool r = true;
#pragma unroll
    for (int k = 0; k < NT / BBC_WAVE; ++k) r = r && red[k] != 0;
    return r;
  }
}
template <int NT>
__device__ __forceinline__ bool blk_any(bool p) {
  return !blk_all<NT>(!p);
}
template <int NT, class T>
__device__ __forceinline__ T blk_min(T v) {
  if constexpr (NT == BBC_WAVE) {
    return wave_min(v);
  } else if constexpr (NT < BBC_WAVE) {
#pragma unroll
    for (int m = NT / 2; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, BBC_WAVE));
    return v;
  } else {
    __shared__ T red[NT / BBC_WAVE];
    const T w = wave_min(v);
    __syncthreads();
    if ((threadIdx.x % BBC_WAVE) == 0) red[threadIdx.x / BBC_WAVE] = w;
    __syncthreads();
    T r = red[0];
#pragma unroll
    for (int k = 1; k < NT / BBC_WAVE; ++k) r = min(r, red[k]);
    return r;
  }
}
template <int NT, class T>
__device__ __forceinline__ T blk_max(T v) {
  return -blk_min<NT>(-v);
}

__device__ __forceinline__ float fmin_nan_safe(float a, float b) { return a < b ? a : b; }

}  // namespace bbc
