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

// Loads per thread issued together before their adds (the partials are
// L2 round trips; one at a time they dominate the small solver kernels).
constexpr int kPartLoads = 8;

// Sum of n partials, identical (same order) in every work-group that asks:
// thread t adds part[t], part[t + 256], ... in increasing order, then the
// block sum combines the threads.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n, double* red) {
  double v = 0.0;
  for (int i0 = threadIdx.x; i0 < n; i0 += kPartLoads * kBlock) {
    double t[kPartLoads];
#pragma unroll
    for (int u = 0; u < kPartLoads; ++u) t[u] = i0 + u * kBlock < n ? part[i0 + u * kBlock] : 0.0;
#pragma unroll
    for (int u = 0; u < kPartLoads; ++u)
      if (i0 + u * kBlock < n) v += t[u];
  }
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
  for (int i0 = threadIdx.x; i0 < nmax; i0 += kPartLoads * kBlock) {
    double t[N][kPartLoads];
#pragma unroll
    for (int u = 0; u < kPartLoads; ++u)
#pragma unroll
      for (int j = 0; j < N; ++j) t[j][u] = i0 + u * kBlock < n[j] ? part[j][i0 + u * kBlock] : 0.0;
#pragma unroll
    for (int u = 0; u < kPartLoads; ++u)
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (i0 + u * kBlock < n[j]) v[j] += t[j][u];
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
