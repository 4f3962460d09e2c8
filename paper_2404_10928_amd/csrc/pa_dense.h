// Internal launch interface of the dense-matrix path (pa_dense.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "pa.h"

namespace pa {

// Row stride of the dense matrix: P rounded up to a multiple of 32 elements.
int64_t dense_ld(int64_t P);

// Shape of the transposed product's partial sums: nchunks row chunks of
// rows_per_chunk rows, each leaving one FP64 partial row of ld entries.
struct DenseShape {
  int64_t ld;
  int col_blocks;
  int64_t nchunks, rows_per_chunk;
};
DenseShape dense_shape(int64_t P, int64_t M);

// A := the dense matrix of g (M * ld elements, padding columns zero)
hipError_t launch_dense_build(const pa_geometry* g, pa_dtype dt, void* a, hipStream_t st);
// y := A x
hipError_t launch_dense_forward(const pa_geometry* g, pa_dtype dt, const void* a, const void* x, void* y,
                                hipStream_t st);
// x := A^T y through nchunks * ld FP64 partials in workspace
hipError_t launch_dense_adjoint(const pa_geometry* g, pa_dtype dt, const void* a, const void* y, void* x,
                                void* workspace, hipStream_t st);

}  // namespace pa
