// Device helpers: NaN-propagating max, wave64 / workgroup reductions, an optimizer barrier.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace tmc {

constexpr int kWave = 64;
constexpr int kMaxWaves = 16;

// v, hidden from the optimizer: values computed from it are not hoisted out of loops
// (keeps loop-invariant address arithmetic from occupying registers across a loop).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// max that returns NaN if either argument is NaN (fmax would drop it).
template <typename T>
__device__ __forceinline__ T nan_max(T a, T b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o, kWave));
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Workgroup reductions; every thread gets the result.  `red` holds kMaxWaves values.
template <typename T>
__device__ __forceinline__ T block_max(T v, T* red) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if ((threadIdx.x % kWave) == 0) red[w] = v;
  __syncthreads();
  T r = red[0];
  for (int i = 1; i < nw; ++i) r = nan_max(r, red[i]);
  return r;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if ((threadIdx.x % kWave) == 0) red[w] = v;
  __syncthreads();
  T r = red[0];
  for (int i = 1; i < nw; ++i) r += red[i];
  return r;
}

__device__ __forceinline__ float fast_exp(float x) { return __expf(x); }
__device__ __forceinline__ double fast_exp(double x) { return exp(x); }
__device__ __forceinline__ float fast_log(float x) { return __logf(x); }
__device__ __forceinline__ double fast_log(double x) { return log(x); }

}  // namespace tmc
