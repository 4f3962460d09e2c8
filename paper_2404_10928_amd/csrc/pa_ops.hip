// HIP kernels for gfx950: the time-domain photoacoustic operator A (scatter
// into LDS time-bin histograms), its adjoint A^T (gather from LDS-staged trace
// windows), and the BLAS-1 / reduction kernels of the CGLS loop.
//
// Operator (time-domain measurement matrix, Eq. 6, with the 1/R of Eq. 7 and
// a unit-peak hat on the sample grid): for pixel p and sensor s,
//   R = max(|r_p - r_s|, r_min), tau = R / (c dt) - t0 / dt,
//   k0 = floor(tau), f = tau - k0, taps (k0, 1 - f) and (k0 + 1, f), weight 1 / R.
//
// Both operators evaluate (k0, f, 1/R) with the same device function on the
// same operand values, so in every precision A^T is the transpose of A up to
// the order of the sums.
#include <hip/hip_runtime.h>

#include "pa_kernels.h"
#include "pa_ops_dev.h"

namespace pa {

// ---------------------------------------------------------------------------
// Single-frame kernels.  Work-group IDs are remapped so each XCD gets a
// contiguous run of tiles (neighbouring tiles read overlapping windows).

template <typename T, int ND, bool FRAC, bool CG>
__global__ void __launch_bounds__(kBlock) bp_kernel(OpParams P, const T* __restrict__ y, T* __restrict__ out,
                                                     T* __restrict__ xcg, const T* __restrict__ pcg,
                                                     const double* __restrict__ alpha, double lambda,
                                                     double* __restrict__ part_s, double* __restrict__ part_x) {
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  bp_body<T, ND, FRAC, CG>(P, tile, tile, y, out, xcg, pcg, alpha, lambda, part_s, part_x);
}

template <typename T, int ND, bool FRAC>
__global__ void __launch_bounds__(kBlock) fp_kernel(OpParams P, const T* __restrict__ x, T* __restrict__ rows,
                                                     int* __restrict__ klo_tab) {
  fp_body<T, ND, FRAC>(P, xcd_remap(blockIdx.x, gridDim.x), x, rows, klo_tab);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) fp_gather_kernel(OpParams P, const T* __restrict__ rows,
                                                            const int* __restrict__ klo_tab, T* __restrict__ y,
                                                            double* __restrict__ part_q) {
  gather_body<T>(P, blockIdx.x, blockIdx.x, rows, klo_tab, y, part_q);
}

// ---------------------------------------------------------------------------
// Launchers.

namespace {

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T, int ND, bool FRAC, bool CG>
hipError_t launch_bp_t(const Plan& pl, const T* y, T* out, const CgArgs* cg, hipStream_t st) {
  const OpParams& P = pl.op;
  auto kern = bp_kernel<T, ND, FRAC, CG>;
  hipError_t e = allow_lds(kern, pl.bp_lds);
  if (e != hipSuccess) return e;
  if (CG)
    kern<<<pl.bp_grid, kBlock, pl.bp_lds, st>>>(P, y, out, static_cast<T*>(cg->x), static_cast<const T*>(cg->p),
                                               cg->alpha, cg->lambda, cg->part_s, cg->part_x);
  else
    kern<<<pl.bp_grid, kBlock, pl.bp_lds, st>>>(P, y, out, nullptr, nullptr, nullptr, 0.0, nullptr, nullptr);
  return hipGetLastError();
}

template <typename T, int ND, bool CG>
hipError_t launch_bp_f(const Plan& pl, const T* y, T* out, const CgArgs* cg, hipStream_t st) {
  return pl.op.t0f != 0.0f ? launch_bp_t<T, ND, true, CG>(pl, y, out, cg, st)
                           : launch_bp_t<T, ND, false, CG>(pl, y, out, cg, st);
}

template <typename T, int ND, bool FRAC>
hipError_t launch_fp_t(const Plan& pl, const T* x, T* rows, int* klo_tab, hipStream_t st) {
  auto kern = fp_kernel<T, ND, FRAC>;
  hipError_t e = allow_lds(kern, pl.fp_lds);
  if (e != hipSuccess) return e;
  kern<<<pl.fp_grid, kBlock, pl.fp_lds, st>>>(pl.op, x, rows, klo_tab);
  return hipGetLastError();
}

template <typename T, int ND>
hipError_t launch_fp_f(const Plan& pl, const T* x, T* rows, int* klo_tab, hipStream_t st) {
  return pl.op.t0f != 0.0f ? launch_fp_t<T, ND, true>(pl, x, rows, klo_tab, st)
                           : launch_fp_t<T, ND, false>(pl, x, rows, klo_tab, st);
}

template <typename T>
hipError_t launch_forward_t(const Plan& pl, const T* x, T* y, void* scratch, double* part_q, hipStream_t st) {
  unsigned char* sc = static_cast<unsigned char*>(scratch);
  T* rows = reinterpret_cast<T*>(sc + pl.part_rows_off);
  int* tab = reinterpret_cast<int*>(sc + pl.klo_tab_off);
  hipError_t e = pl.ndim == 2 ? launch_fp_f<T, 2>(pl, x, rows, tab, st) : launch_fp_f<T, 3>(pl, x, rows, tab, st);
  if (e != hipSuccess) return e;
  auto g = fp_gather_kernel<T>;
  if ((e = allow_lds(g, pl.gather_lds)) != hipSuccess) return e;
  g<<<pl.gather_grid, kBlock, pl.gather_lds, st>>>(pl.op, rows, tab, y, part_q);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint(const Plan& pl, const void* y, void* x, const CgArgs* cg, hipStream_t st) {
  if (pl.bp_grid == 0) return hipSuccess;
  const bool CGm = cg != nullptr;
  if (pl.dtype == PA_F32) {
    auto yy = static_cast<const float*>(y);
    auto xx = static_cast<float*>(x);
    if (pl.ndim == 2) return CGm ? launch_bp_f<float, 2, true>(pl, yy, xx, cg, st) : launch_bp_f<float, 2, false>(pl, yy, xx, cg, st);
    return CGm ? launch_bp_f<float, 3, true>(pl, yy, xx, cg, st) : launch_bp_f<float, 3, false>(pl, yy, xx, cg, st);
  }
  auto yy = static_cast<const double*>(y);
  auto xx = static_cast<double*>(x);
  if (pl.ndim == 2) return CGm ? launch_bp_f<double, 2, true>(pl, yy, xx, cg, st) : launch_bp_f<double, 2, false>(pl, yy, xx, cg, st);
  return CGm ? launch_bp_f<double, 3, true>(pl, yy, xx, cg, st) : launch_bp_f<double, 3, false>(pl, yy, xx, cg, st);
}

hipError_t launch_forward(const Plan& pl, const void* x, void* y, void* scratch, double* part_q, hipStream_t st) {
  if (pl.fp_grid == 0) {
    // nothing to scatter: y = 0, ||y||^2 = 0
    hipError_t e = launch_fill(pl.dtype, y, pl.M, st);
    if (e != hipSuccess || !part_q) return e;
    return launch_fill(PA_F64, part_q, 1, st);
  }
  if (pl.dtype == PA_F32)
    return launch_forward_t<float>(pl, static_cast<const float*>(x), static_cast<float*>(y), scratch, part_q, st);
  return launch_forward_t<double>(pl, static_cast<const double*>(x), static_cast<double*>(y), scratch, part_q, st);
}

}  // namespace pa
