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

// N fixed-order sums of partials in one pass: the loads of all N arrays are
// in flight together and the block reduction runs once, yet out[j] is
// bit-identical to sum_partials(part[j], n[j], .) (same per-thread order,
// same shuffle tree, same combination of the four waves).  red: 4 N doubles.
template <int N>
__device__ __forceinline__ void sum_partials_n(const double* const (&part)[N], const int (&n)[N], double (&out)[N],
                                               double* red) {
  double v[N];
  int nmax = 0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    v[j] = 0.0;
    nmax = n[j] > nmax ? n[j] : nmax;
  }
  for (int i = threadIdx.x; i < nmax; i += kBlock) {
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (i < n[j]) v[j] += part[j][i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] += __shfl_xor(v[j], o, 64);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) red[4 * j + (threadIdx.x >> 6)] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) out[j] = (red[4 * j + 0] + red[4 * j + 1]) + (red[4 * j + 2] + red[4 * j + 3]);
}

}  // namespace dev
}  // namespace pa
