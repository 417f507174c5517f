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
// FP32 and FP64 minima and maxima over the wave through DPP moves (VALU, no
// LDS round trip): butterflies within each row of 16 lanes (quad_perm
// [1,0,3,2], quad_perm [2,3,0,1], half-row mirror, row mirror), then the four
// row results through readlane.  Every lane gets the result; all 64 lanes
// must be active.  min and max are exact, so the result does not depend on
// the order in which the lanes are combined.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(x >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(x), l), hi = __builtin_amdgcn_readlane(int(x >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <bool MAX, class T>
__device__ __forceinline__ T wave_minmax_dpp(T v) {
  auto op = [](T a, T b) { return MAX ? max(a, b) : min(a, b); };
  v = op(v, dpp_mov<0xB1>(v));
  v = op(v, dpp_mov<0x4E>(v));
  v = op(v, dpp_mov<0x141>(v));
  v = op(v, dpp_mov<0x140>(v));
  return op(op(read_lane(v, 0), read_lane(v, 16)), op(read_lane(v, 32), read_lane(v, 48)));
}
template <>
__device__ __forceinline__ double wave_min<double>(double v) {
  return wave_minmax_dpp<false>(v);
}
template <>
__device__ __forceinline__ double wave_max<double>(double v) {
  return wave_minmax_dpp<true>(v);
}
template <>
__device__ __forceinline__ float wave_min<float>(float v) {
  return wave_minmax_dpp<false>(v);
}
template <>
__device__ __forceinline__ float wave_max<float>(float v) {
  return wave_minmax_dpp<true>(v);
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
