// Batched operator kernels: one launch covers every frame of a batch.  Each
// work-group finds its frame in the device frame table and runs the same
// device body as the single-frame kernels with that frame's plan, so every
// frame's result equals its single-frame result.
#include <hip/hip_runtime.h>

#include "pa_kernels.h"
#include "pa_ops_dev.h"

namespace pa {

template <typename T, typename PH, int ND, bool FRAC, bool CG>
__global__ void __launch_bounds__(kBlock) bp_batched(const FrameDesc* __restrict__ B, int nf, const T* __restrict__ y,
                                                      T* __restrict__ out, T* __restrict__ xcg,
                                                      const T* __restrict__ pcg, const double* __restrict__ alpha,
                                                      int astride, int acol, double lambda,
                                                      double* __restrict__ part_s, double* __restrict__ part_x) {
  const int g = xcd_remap(blockIdx.x, gridDim.x);
  const int f = find_frame<&FrameDesc::b_bp>(B, nf, g);
  const FrameDesc& F = B[f];
  const int tile = g - F.b_bp;
  bp_body<T, PH, ND, FRAC, CG>(F.op, tile, F.s_bp + tile, y + F.yo, out + F.xo, CG ? xcg + F.xo : nullptr,
                               CG ? pcg + F.xo : nullptr, CG ? alpha + (size_t)F.frame * astride + acol : nullptr,
                               lambda, part_s, part_x);
}

template <typename T, typename PH, int ND, bool FRAC, bool FIX>
__global__ void __launch_bounds__(kBlock) fp_batched(const FrameDesc* __restrict__ B, int nf, const T* __restrict__ x,
                                                      T* __restrict__ y, double* __restrict__ part_q) {
  const int g = blockIdx.x;
  const int f = find_frame<&FrameDesc::b_fp>(B, nf, g);
  const FrameDesc& F = B[f];
  const int local = g - F.b_fp;
  fp_body<T, PH, ND, FRAC, FIX>(F.op, local, F.s_fp + local, x + F.xo, y + F.yo, part_q);
}

namespace {

template <typename K>
hipError_t allow_lds_b(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T, typename PH, int ND, bool FRAC, bool CG>
hipError_t bp_b(const BatchLaunch& L, const T* y, T* out, const BatchCg* cg, hipStream_t st) {
  auto kern = bp_batched<T, PH, ND, FRAC, CG>;
  hipError_t e = allow_lds_b(kern, L.bp_lds);
  if (e != hipSuccess) return e;
  kern<<<L.bp_grid, kBlock, L.bp_lds, st>>>(L.table, L.nf, y, out, CG ? static_cast<T*>(cg->x) : nullptr,
                                            CG ? static_cast<const T*>(cg->p) : nullptr, CG ? cg->alpha : nullptr,
                                            CG ? cg->astride : 0, CG ? cg->acol : 0, CG ? cg->lambda : 0.0,
                                            CG ? cg->part_s : nullptr, CG ? cg->part_x : nullptr);
  return hipGetLastError();
}

template <typename T, typename PH, int ND>
hipError_t bp_bf(const BatchLaunch& L, const void* y, void* out, const BatchCg* cg, hipStream_t st) {
  auto yy = static_cast<const T*>(y);
  auto xx = static_cast<T*>(out);
  if (cg) return L.frac ? bp_b<T, PH, ND, true, true>(L, yy, xx, cg, st) : bp_b<T, PH, ND, false, true>(L, yy, xx, cg, st);
  return L.frac ? bp_b<T, PH, ND, true, false>(L, yy, xx, cg, st) : bp_b<T, PH, ND, false, false>(L, yy, xx, cg, st);
}

template <typename T, typename PH, int ND, bool FRAC, bool FIX>
hipError_t fwd_b(const BatchLaunch& L, const T* x, T* y, double* part_q, hipStream_t st) {
  auto k = fp_batched<T, PH, ND, FRAC, FIX>;
  hipError_t e = allow_lds_b(k, L.fp_lds);
  if (e != hipSuccess) return e;
  k<<<L.fp_grid, kBlock, L.fp_lds, st>>>(L.table, L.nf, x, y, part_q);
  return hipGetLastError();
}

template <typename T, typename PH, int ND>
hipError_t fwd_bf(const BatchLaunch& L, const void* x, void* y, double* part_q, hipStream_t st) {
  auto xx = static_cast<const T*>(x);
  auto yy = static_cast<T*>(y);
  if constexpr (sizeof(PH) == 4) {
    if (L.ffix) return L.frac ? fwd_b<T, PH, ND, true, true>(L, xx, yy, part_q, st) : fwd_b<T, PH, ND, false, true>(L, xx, yy, part_q, st);
  }
  return L.frac ? fwd_b<T, PH, ND, true, false>(L, xx, yy, part_q, st) : fwd_b<T, PH, ND, false, false>(L, xx, yy, part_q, st);
}

template <typename T, typename PH>
hipError_t adj_bd(const BatchLaunch& L, const void* y, void* x, const BatchCg* cg, hipStream_t st) {
  return L.ndim == 2 ? bp_bf<T, PH, 2>(L, y, x, cg, st) : bp_bf<T, PH, 3>(L, y, x, cg, st);
}

template <typename T, typename PH>
hipError_t fwd_bd(const BatchLaunch& L, const void* x, void* y, double* part_q, hipStream_t st) {
  return L.ndim == 2 ? fwd_bf<T, PH, 2>(L, x, y, part_q, st) : fwd_bf<T, PH, 3>(L, x, y, part_q, st);
}

}  // namespace

hipError_t launch_adjoint_batched(const BatchLaunch& L, const void* y, void* x, const BatchCg* cg, hipStream_t st) {
  if (L.bp_grid == 0) return hipSuccess;
  switch (L.dtype) {
    case PA_F32: return adj_bd<float, float>(L, y, x, cg, st);
    case PA_MIXED: return adj_bd<double, float>(L, y, x, cg, st);
    default: return adj_bd<double, double>(L, y, x, cg, st);
  }
}

hipError_t launch_forward_batched(const BatchLaunch& L, const void* x, void* y, double* part_q, hipStream_t st) {
  if (L.fp_grid == 0) return hipSuccess;  // no frame has samples
  switch (L.dtype) {
    case PA_F32: return fwd_bd<float, float>(L, x, y, part_q, st);
    case PA_MIXED: return fwd_bd<double, float>(L, x, y, part_q, st);
    default: return fwd_bd<double, double>(L, x, y, part_q, st);
  }
}

}  // namespace pa
