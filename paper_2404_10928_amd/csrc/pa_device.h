// Device helpers shared by the operator and solver kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "pa_plan.h"

namespace pa {
namespace dev {

// Wave-then-block FP64 sum in a fixed order; every thread gets the total.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Sum of n partials, identical (same order) in every work-group that asks.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) v += part[i];
  return block_sum(v, red);
}

}  // namespace dev
}  // namespace pa
