// Block reductions of the FP64 vector kernels (256 threads, 64-wide waves).
// Sums are taken in a fixed order, so results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

namespace ts {

constexpr int RT = 256;  // threads per block of the vector kernels

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  return v;
}

// Sum over the block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[RT / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < RT / 64; ++i) s += sh[i];
  return s;
}

// Fixed-order sum of kRedBlocks partials in one block; valid in thread 0.
__device__ __forceinline__ double sum_partials(const double* partial, int count) {
  double a = 0.0;
  for (int i = threadIdx.x; i < count; i += RT) a += partial[i];
  return block_sum(a);
}

}  // namespace ts
