// Batched operator kernels: one launch covers every frame of a batch.  Each
// work-group finds its frame in the device frame table and runs the same
// device body as the single-frame kernels with that frame's plan, so every
// frame's result equals its single-frame result.
#include <hip/hip_runtime.h>

#include "pa_kernels.h"
#include "pa_ops_dev.h"

namespace pa {

template <typename T, int ND, bool FRAC, bool CG>
__global__ void __launch_bounds__(kBlock) bp_batched(const FrameDesc* __restrict__ B, int nf, const T* __restrict__ y,
                                                      T* __restrict__ out, T* __restrict__ xcg,
                                                      const T* __restrict__ pcg, const double* __restrict__ alpha,
                                                      int astride, int acol, double lambda,
                                                      double* __restrict__ part_s, double* __restrict__ part_x) {
  const int g = xcd_remap(blockIdx.x, gridDim.x);
  const int f = find_frame<&FrameDesc::b_bp>(B, nf, g);
  const FrameDesc& F = B[f];
  const int tile = g - F.b_bp;
  bp_body<T, ND, FRAC, CG>(F.op, tile, F.s_bp + tile, y + F.yo, out + F.xo, CG ? xcg + F.xo : nullptr,
                           CG ? pcg + F.xo : nullptr, CG ? alpha + (size_t)F.frame * astride + acol : nullptr, lambda,
                           part_s, part_x);
}

template <typename T, int ND, bool FRAC>
__global__ void __launch_bounds__(kBlock) fp_batched(const FrameDesc* __restrict__ B, int nf, const T* __restrict__ x,
                                                      unsigned char* __restrict__ scratch) {
  const int g = xcd_remap(blockIdx.x, gridDim.x);
  const int f = find_frame<&FrameDesc::b_fp>(B, nf, g);
  const FrameDesc& F = B[f];
  fp_body<T, ND, FRAC>(F.op, g - F.b_fp, x + F.xo, reinterpret_cast<T*>(scratch + F.scr),
                       reinterpret_cast<int*>(scratch + F.scr_tab));
}

template <typename T>
__global__ void __launch_bounds__(kBlock) gather_batched(const FrameDesc* __restrict__ B, int nf,
                                                          const unsigned char* __restrict__ scratch, T* __restrict__ y,
                                                          double* __restrict__ part_q) {
  const int g = blockIdx.x;
  const int f = find_frame<&FrameDesc::b_ga>(B, nf, g);
  const FrameDesc& F = B[f];
  const int local = g - F.b_ga;
  if (F.n_fp == 0) {  // a frame without pixels: y = 0
    const int s = local / F.op.nseg, k0 = (local - s * F.op.nseg) * F.op.kseg;
    const int kn = min(F.op.kseg, F.op.K - k0);
    for (int i = threadIdx.x; i < kn; i += kBlock) y[F.yo + (size_t)s * F.op.K + k0 + i] = (T)0;
    if (part_q && threadIdx.x == 0) part_q[F.s_ga + local] = 0.0;
    return;
  }
  gather_body<T>(F.op, local, F.s_ga + local, reinterpret_cast<const T*>(scratch + F.scr),
                 reinterpret_cast<const int*>(scratch + F.scr_tab), y + F.yo, part_q);
}

namespace {

template <typename K>
hipError_t allow_lds_b(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T, int ND, bool FRAC, bool CG>
hipError_t bp_b(const BatchLaunch& L, const T* y, T* out, const BatchCg* cg, hipStream_t st) {
  auto kern = bp_batched<T, ND, FRAC, CG>;
  hipError_t e = allow_lds_b(kern, L.bp_lds);
  if (e != hipSuccess) return e;
  kern<<<L.bp_grid, kBlock, L.bp_lds, st>>>(L.table, L.nf, y, out, CG ? static_cast<T*>(cg->x) : nullptr,
                                            CG ? static_cast<const T*>(cg->p) : nullptr, CG ? cg->alpha : nullptr,
                                            CG ? cg->astride : 0, CG ? cg->acol : 0, CG ? cg->lambda : 0.0,
                                            CG ? cg->part_s : nullptr, CG ? cg->part_x : nullptr);
  return hipGetLastError();
}

template <typename T, int ND, bool CG>
hipError_t bp_bf(const BatchLaunch& L, const T* y, T* out, const BatchCg* cg, hipStream_t st) {
  return L.frac ? bp_b<T, ND, true, CG>(L, y, out, cg, st) : bp_b<T, ND, false, CG>(L, y, out, cg, st);
}

template <typename T, int ND>
hipError_t fwd_b(const BatchLaunch& L, const T* x, T* y, double* part_q, hipStream_t st) {
  hipError_t e;
  if (L.fp_grid > 0) {
    if (L.frac) {
      auto k = fp_batched<T, ND, true>;
      if ((e = allow_lds_b(k, L.fp_lds)) != hipSuccess) return e;
      k<<<L.fp_grid, kBlock, L.fp_lds, st>>>(L.table, L.nf, x, L.scratch);
    } else {
      auto k = fp_batched<T, ND, false>;
      if ((e = allow_lds_b(k, L.fp_lds)) != hipSuccess) return e;
      k<<<L.fp_grid, kBlock, L.fp_lds, st>>>(L.table, L.nf, x, L.scratch);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (L.gather_grid > 0) {
    auto k = gather_batched<T>;
    if ((e = allow_lds_b(k, L.gather_lds)) != hipSuccess) return e;
    k<<<L.gather_grid, kBlock, L.gather_lds, st>>>(L.table, L.nf, L.scratch, y, part_q);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_adjoint_batched(const BatchLaunch& L, const void* y, void* x, const BatchCg* cg, hipStream_t st) {
  if (L.bp_grid == 0) return hipSuccess;
  const bool CGm = cg != nullptr;
  if (L.dtype == PA_F32) {
    auto yy = static_cast<const float*>(y);
    auto xx = static_cast<float*>(x);
    if (L.ndim == 2) return CGm ? bp_bf<float, 2, true>(L, yy, xx, cg, st) : bp_bf<float, 2, false>(L, yy, xx, cg, st);
    return CGm ? bp_bf<float, 3, true>(L, yy, xx, cg, st) : bp_bf<float, 3, false>(L, yy, xx, cg, st);
  }
  auto yy = static_cast<const double*>(y);
  auto xx = static_cast<double*>(x);
  if (L.ndim == 2) return CGm ? bp_bf<double, 2, true>(L, yy, xx, cg, st) : bp_bf<double, 2, false>(L, yy, xx, cg, st);
  return CGm ? bp_bf<double, 3, true>(L, yy, xx, cg, st) : bp_bf<double, 3, false>(L, yy, xx, cg, st);
}

hipError_t launch_forward_batched(const BatchLaunch& L, const void* x, void* y, double* part_q, hipStream_t st) {
  if (L.dtype == PA_F32) {
    auto xx = static_cast<const float*>(x);
    auto yy = static_cast<float*>(y);
    return L.ndim == 2 ? fwd_b<float, 2>(L, xx, yy, part_q, st) : fwd_b<float, 3>(L, xx, yy, part_q, st);
  }
  auto xx = static_cast<const double*>(x);
  auto yy = static_cast<double*>(y);
  return L.ndim == 2 ? fwd_b<double, 2>(L, xx, yy, part_q, st) : fwd_b<double, 3>(L, xx, yy, part_q, st);
}

}  // namespace pa
