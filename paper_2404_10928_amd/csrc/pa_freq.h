// Internal launch interface of the frequency-domain operator (pa_freq.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "pa.h"

namespace pa {

// Chunking of both products and the FP64 workspace their partial sums need.
struct FreqShape {
  int fwd_fblocks;        // blocks of 256 frequencies
  int64_t fwd_chunk_px;   // pixels per forward work-group
  int fwd_chunks;         // pixel chunks (forward partial sums per output)
  int adj_pblocks;        // blocks of 256 pixels
  int adj_sens;           // sensors per adjoint work-group
  int adj_chunks;         // sensor chunks (adjoint partial sums per pixel)
  size_t workspace;       // bytes
};
FreqShape freq_shape(int64_t P, int32_t S, int32_t nf);

// Y := K x, Y complex interleaved [S][nf][2]
hipError_t launch_freq_forward(const pa_geometry* g, pa_dtype dt, double f0, double df, int32_t nf, const void* x,
                               void* Y, void* workspace, hipStream_t st);
// x := Re(K^H Y)
hipError_t launch_freq_adjoint(const pa_geometry* g, pa_dtype dt, double f0, double df, int32_t nf, const void* Y,
                               void* x, void* workspace, hipStream_t st);

}  // namespace pa
