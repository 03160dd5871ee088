// Wavefront (64 lanes) and block reductions with a fixed combination order,
// so every reduction in the library is deterministic run to run.
#pragma once

#include <hip/hip_runtime.h>

namespace rt {

constexpr int kWave = 64;

// Sum over aligned groups of G lanes (G a power of two <= 64); every lane of
// the group receives the group total.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

template <int G, typename T>
__device__ __forceinline__ T group_max(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, G);
    v = v > w ? v : w;
  }
  return v;
}

// Block-wide sum of one value per thread; result valid in thread 0.
// `sh` must hold blockDim.x / 64 elements.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  v = group_sum<kWave>(v);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T out = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) out += sh[i];
  }
  __syncthreads();
  return out;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T* sh) {
  v = group_max<kWave>(v);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T out = sh[0];
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x / kWave); ++i) out = out > sh[i] ? out : sh[i];
  }
  __syncthreads();
  return out;
}

}  // namespace rt
