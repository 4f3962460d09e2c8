// Internal launch interface between the C ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "pa_plan.h"

namespace pa {

// Arguments of the adjoint's CGLS epilogue: x += (*alpha) p;
// out = A^T r - lambda x; per-work-group FP64 sums of ||out||^2 and ||x||^2.
struct CgArgs {
  void* x;
  const void* p;
  const double* alpha;
  double lambda;
  double* part_s;
  double* part_x;
};

hipError_t launch_fill(pa_dtype dt, void* p, int64_t n, hipStream_t st);
// x := A^T y (or the CGLS epilogue when cg != nullptr)
hipError_t launch_adjoint(const Plan& pl, const void* y, void* x, const CgArgs* cg, hipStream_t st);
// y := A x in two passes through `scratch` (plan.fwd_scratch bytes); when
// part_q is not NULL it receives plan.gather_grid FP64 partial sums of ||y||^2
hipError_t launch_forward(const Plan& pl, const void* x, void* y, void* scratch, double* part_q, hipStream_t st);
hipError_t launch_init_r(pa_dtype dt, void* r, const void* y, const void* q, int64_t m, double* part_r, int* status,
                         double* alpha0, hipStream_t st);
hipError_t launch_upd_r(pa_dtype dt, void* r, const void* q, int64_t m, const double* part_q, int gq, const double* part_p,
                        int gp, double lambda, const double* gamma_k, double* alpha_k, int* status, int k, double* part_r,
                        hipStream_t st);
hipError_t launch_dir(pa_dtype dt, void* p, const void* s, int64_t np, void* q, int64_t m, const double* part_s, int gs,
                      const double* part_x, int gx, const double* part_r, int gr, double lambda, double* gamma, int k,
                      const int* status, double* hist, double* part_p, hipStream_t st);

}  // namespace pa
