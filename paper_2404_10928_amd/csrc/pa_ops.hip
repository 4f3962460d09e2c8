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
// Single-frame kernels.  T is the element type of the vectors, PH the type of
// the per-pair delay arithmetic (PA_F32: float/float, PA_F64: double/double,
// PA_MIXED: double/float).  Adjoint work-group IDs are remapped so each XCD
// gets a contiguous run of tiles (neighbouring tiles read overlapping windows).

template <typename T, typename PH, int ND, bool FRAC, bool CG>
__global__ void __launch_bounds__(kBlock) bp_kernel(OpParams P, const T* __restrict__ y, T* __restrict__ out,
                                                     T* __restrict__ xcg, const T* __restrict__ pcg,
                                                     const double* __restrict__ alpha, double lambda,
                                                     double* __restrict__ part_s, double* __restrict__ part_x) {
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  bp_body<T, PH, ND, FRAC, CG>(P, tile, tile, y, out, xcg, pcg, alpha, lambda, part_s, part_x);
}

template <typename T, typename PH, int ND, bool FRAC, bool FIX>
__global__ void __launch_bounds__(kBlock) fp_kernel(OpParams P, const T* __restrict__ x, T* __restrict__ y,
                                                     double* __restrict__ part_q) {
  fp_body<T, PH, ND, FRAC, FIX>(P, blockIdx.x, blockIdx.x, x, y, part_q);
}

// Its LDS (about 39 KiB at the 512x512 workload) admits four work-groups, so
// four waves per SIMD, per CU: telling the compiler so lets it use up to 128
// VGPRs for the interleaved pixel chains instead of aiming at eight waves.
template <int ND, bool FRAC, bool CG>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 4)))
fp2_kernel(OpParams P, const float* __restrict__ x, float* __restrict__ rows, int* __restrict__ klo_tab, CgDirArgs cg) {
  fp2_body<ND, FRAC, CG>(P, xcd_remap(blockIdx.x, gridDim.x), x, rows, klo_tab, cg);
}

__global__ void __launch_bounds__(kBlock) fp_gather_kernel(OpParams P, const float* __restrict__ rows,
                                                            const int* __restrict__ klo_tab, float* __restrict__ y,
                                                            double* __restrict__ part_q) {
  gather_body(P, xcd_remap(blockIdx.x, gridDim.x), blockIdx.x, rows, klo_tab, y, part_q);
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

template <typename T, typename PH, int ND, bool FRAC, bool CG>
hipError_t launch_bp_t(const Plan& pl, const T* y, T* out, const CgArgs* cg, hipStream_t st) {
  const OpParams& P = pl.op;
  auto kern = bp_kernel<T, PH, ND, FRAC, CG>;
  hipError_t e = allow_lds(kern, pl.bp_lds);
  if (e != hipSuccess) return e;
  if (CG)
    kern<<<pl.bp_grid, kBlock, pl.bp_lds, st>>>(P, y, out, static_cast<T*>(cg->x), static_cast<const T*>(cg->p),
                                               cg->alpha, cg->lambda, cg->part_s, cg->part_x);
  else
    kern<<<pl.bp_grid, kBlock, pl.bp_lds, st>>>(P, y, out, nullptr, nullptr, nullptr, 0.0, nullptr, nullptr);
  return hipGetLastError();
}

template <typename T, typename PH, int ND>
hipError_t launch_bp_f(const Plan& pl, const void* y, void* out, const CgArgs* cg, hipStream_t st) {
  auto yy = static_cast<const T*>(y);
  auto xx = static_cast<T*>(out);
  const bool frac = pl.op.t0f != 0.0f;
  if (cg) return frac ? launch_bp_t<T, PH, ND, true, true>(pl, yy, xx, cg, st) : launch_bp_t<T, PH, ND, false, true>(pl, yy, xx, cg, st);
  return frac ? launch_bp_t<T, PH, ND, true, false>(pl, yy, xx, cg, st) : launch_bp_t<T, PH, ND, false, false>(pl, yy, xx, cg, st);
}

template <typename T, typename PH, int ND, bool FRAC, bool FIX>
hipError_t launch_fp_t(const Plan& pl, const T* x, T* y, double* part_q, hipStream_t st) {
  auto kern = fp_kernel<T, PH, ND, FRAC, FIX>;
  hipError_t e = allow_lds(kern, pl.fp_lds);
  if (e != hipSuccess) return e;
  kern<<<pl.fp_grid, kBlock, pl.fp_lds, st>>>(pl.op, x, y, part_q);
  return hipGetLastError();
}

template <typename T, typename PH, int ND>
hipError_t launch_fp_f(const Plan& pl, const void* x, void* y, double* part_q, hipStream_t st) {
  auto xx = static_cast<const T*>(x);
  auto yy = static_cast<T*>(y);
  const bool frac = pl.op.t0f != 0.0f;
  if constexpr (sizeof(PH) == 4) {
    if (pl.op.ffix)
      return frac ? launch_fp_t<T, PH, ND, true, true>(pl, xx, yy, part_q, st)
                  : launch_fp_t<T, PH, ND, false, true>(pl, xx, yy, part_q, st);
  }
  return frac ? launch_fp_t<T, PH, ND, true, false>(pl, xx, yy, part_q, st)
              : launch_fp_t<T, PH, ND, false, false>(pl, xx, yy, part_q, st);
}

template <typename T, typename PH>
hipError_t launch_adj_d(const Plan& pl, const void* y, void* x, const CgArgs* cg, hipStream_t st) {
  return pl.ndim == 2 ? launch_bp_f<T, PH, 2>(pl, y, x, cg, st) : launch_bp_f<T, PH, 3>(pl, y, x, cg, st);
}

template <typename T, typename PH>
hipError_t launch_fwd_d(const Plan& pl, const void* x, void* y, double* part_q, hipStream_t st) {
  return pl.ndim == 2 ? launch_fp_f<T, PH, 2>(pl, x, y, part_q, st) : launch_fp_f<T, PH, 3>(pl, x, y, part_q, st);
}

template <int ND, bool FRAC, bool CG>
hipError_t launch_fp2_t(const Plan& pl, const float* x, float* rows, int* tab, const CgDirArgs& cg, hipStream_t st) {
  auto kern = fp2_kernel<ND, FRAC, CG>;
  hipError_t e = allow_lds(kern, pl.fp2_lds);
  if (e != hipSuccess) return e;
  kern<<<pl.fp2_grid, kBlock, pl.fp2_lds, st>>>(pl.op, x, rows, tab, cg);
  return hipGetLastError();
}

template <bool CG>
hipError_t launch_fp2_f(const Plan& pl, const float* x, float* rows, int* tab, const CgDirArgs& cg, hipStream_t st) {
  const bool frac = pl.op.t0f != 0.0f;
  if (pl.ndim == 2)
    return frac ? launch_fp2_t<2, true, CG>(pl, x, rows, tab, cg, st) : launch_fp2_t<2, false, CG>(pl, x, rows, tab, cg, st);
  return frac ? launch_fp2_t<3, true, CG>(pl, x, rows, tab, cg, st) : launch_fp2_t<3, false, CG>(pl, x, rows, tab, cg, st);
}

// Pass 1 (with the direction update when cg != nullptr), then pass 2.
hipError_t launch_forward_two_pass(const Plan& pl, const float* x, float* y, void* scratch, double* part_q,
                                   const CgDirArgs* cg, hipStream_t st) {
  unsigned char* sc = static_cast<unsigned char*>(scratch);
  float* rows = reinterpret_cast<float*>(sc + pl.part_rows_off);
  int* tab = reinterpret_cast<int*>(sc + pl.klo_tab_off);
  hipError_t e = cg ? launch_fp2_f<true>(pl, x, rows, tab, *cg, st) : launch_fp2_f<false>(pl, x, rows, tab, CgDirArgs{}, st);
  if (e != hipSuccess) return e;
  fp_gather_kernel<<<pl.gather_grid, kBlock, 0, st>>>(pl.op, rows, tab, y, part_q);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint(const Plan& pl, const void* y, void* x, const CgArgs* cg, hipStream_t st) {
  if (pl.bp_grid == 0) return hipSuccess;
  switch (pl.dtype) {
    case PA_F32: return launch_adj_d<float, float>(pl, y, x, cg, st);
    case PA_MIXED: return launch_adj_d<double, float>(pl, y, x, cg, st);
    default: return launch_adj_d<double, double>(pl, y, x, cg, st);
  }
}

hipError_t launch_forward(const Plan& pl, const void* x, void* y, double* part_q, void* scratch, hipStream_t st) {
  if (pl.fp_grid == 0) {  // no samples: nothing to write, ||y||^2 = 0
    if (!part_q) return hipSuccess;
    return launch_fill(PA_F64, part_q, 1, st);
  }
  if (pl.two_pass && scratch && pl.fwd_scratch > 0)
    return launch_forward_two_pass(pl, static_cast<const float*>(x), static_cast<float*>(y), scratch, part_q, nullptr, st);
  switch (pl.dtype) {
    case PA_F32: return launch_fwd_d<float, float>(pl, x, y, part_q, st);
    case PA_MIXED: return launch_fwd_d<double, float>(pl, x, y, part_q, st);
    default: return launch_fwd_d<double, double>(pl, x, y, part_q, st);
  }
}

hipError_t launch_forward_cg(const Plan& pl, const CgDirArgs& dir, float* q, double* part_q, void* scratch,
                             hipStream_t st) {
  if (!(pl.two_pass && scratch && pl.fwd_scratch > 0 && pl.fp2_grid > 0 && pl.dtype == PA_F32)) return hipErrorInvalidValue;
  return launch_forward_two_pass(pl, nullptr, q, scratch, part_q, &dir, st);
}

}  // namespace pa
