// BLAS-1 and CGLS scalar kernels for gfx950.  Each reduction produces one
// FP64 partial per work-group; consumers add the partials in a fixed order,
// so every scalar of the solve is reproducible run to run.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pa_device.h"
#include "pa_kernels.h"

namespace pa {

using dev::block_sum;
using dev::sum_partials;

// Elements per thread whose loads the CGLS update kernels issue before their
// step-size reductions (the single-frame grids give 4 per thread on the
// image and up to 8 on the traces).
constexpr int kPrefetch = 4;

// ---------------------------------------------------------------------------
// BLAS-1 and CGLS scalar kernels.  Grids are fixed per vector length, so the
// FP64 partial sums are always formed in the same order.

template <typename T>
__global__ void __launch_bounds__(kBlock) fill_kernel(T* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = (T)0;
}

// The bodies below run as work-group `bid` of `nblk`; the single-frame
// kernels pass their own grid, the batched kernels a frame's block range, so
// a frame's partial sums come out identical either way.

// r = y - q (q may be NULL); partial sums of ||r||^2; resets the solve state.
template <typename T>
__device__ __forceinline__ void init_r_body(int bid, int nblk, T* __restrict__ r, const T* __restrict__ y,
                                            const T* __restrict__ q, int64_t m, double* __restrict__ part_r,
                                            int* __restrict__ status, double* __restrict__ alpha0) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)bid * kBlock + threadIdx.x; i < m; i += (int64_t)nblk * kBlock) {
    const double v = q ? (double)y[i] - (double)q[i] : (double)y[i];
    const T t = (T)v;
    r[i] = t;
    acc += (double)t * (double)t;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) {
    part_r[bid] = acc;
    if (bid == 0) {
      *status = -1;
      *alpha0 = 0.0;
    }
  }
}

// delta = ||q||^2 + lambda ||p||^2, alpha = gamma_k / delta (0 once stopped),
// r -= alpha q, partial sums of ||r||^2.
template <typename T>
__device__ __forceinline__ void upd_r_body(int bid, int nblk, T* __restrict__ r, const T* __restrict__ q, int64_t m,
                                           const double* __restrict__ part_q, int gq, const double* __restrict__ part_p,
                                           int gp, double lambda, const double* __restrict__ gamma_k,
                                           double* __restrict__ alpha_k, int* __restrict__ status, int k,
                                           double* __restrict__ part_r) {
  __shared__ double red[8];
  // The first kPrefetch elements' loads go out before the step size is
  // known, so their latency overlaps the partial sums.
  const int64_t stride = (int64_t)nblk * kBlock;
  const int64_t i0 = (int64_t)bid * kBlock + threadIdx.x;
  // (every load is issued, element 0 in place of one past the end, so they
  // go out back to back; the extra values are never used)
  T rv[kPrefetch], qv[kPrefetch];
  if (m > 0) {
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
      const int64_t i = i0 + u * stride;
      rv[u] = r[i < m ? i : 0];
      qv[u] = q[i < m ? i : 0];
    }
  }
  double sums[2];
  dev::sum_partials_n<2>({part_q, part_p}, {gq, gp}, sums, red);
  const double qq = sums[0], pp = sums[1];
  const double delta = qq + lambda * pp;
  const double g = *gamma_k;
  const int st = *status;
  const bool stop = st >= 0 || !(g > 0.0) || !(delta > 0.0) || !isfinite(g) || !isfinite(delta);
  const double a = stop ? 0.0 : g / delta;
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < kPrefetch; ++u) {
    const int64_t i = i0 + u * stride;
    if (i < m) {
      T t = rv[u];
      if (a != 0.0) {
        t = (T)((double)t - a * (double)qv[u]);
        r[i] = t;
      }
      acc += (double)t * (double)t;
    }
  }
  for (int64_t i = i0 + kPrefetch * stride; i < m; i += stride) {
    T t = r[i];
    if (a != 0.0) {
      t = (T)((double)t - a * (double)q[i]);
      r[i] = t;
    }
    acc += (double)t * (double)t;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) {
    part_r[bid] = acc;
    if (bid == 0) {
      *alpha_k = a;
      if (stop && st < 0) *status = k;
    }
  }
}

// gamma_{k+1} = ||s||^2, beta = gamma_{k+1} / gamma_k (0 at the start or once
// stopped), p = s + beta p, q = 0, history row k + 1, partial sums of ||p||^2.
template <typename T>
__device__ __forceinline__ void dir_body(int bid, int nblk, T* __restrict__ p, const T* __restrict__ s, int64_t np,
                                         T* __restrict__ q, int64_t m, const double* __restrict__ part_s, int gs,
                                         const double* __restrict__ part_x, int gx, const double* __restrict__ part_r,
                                         int gr, double lambda, double* __restrict__ gamma, int k,
                                         const int* __restrict__ status, double* __restrict__ hist,
                                         double* __restrict__ part_p) {
  __shared__ double red[12];
  // The first kPrefetch elements' loads go out before beta is known.
  const int64_t stride = (int64_t)nblk * kBlock;
  const int64_t i0 = (int64_t)bid * kBlock + threadIdx.x;
  // (loads issued back to back, as in upd_r_body)
  T sv[kPrefetch], pv[kPrefetch];
  if (np > 0) {
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
      const int64_t i = i0 + u * stride;
      sv[u] = s[i < np ? i : 0];
      pv[u] = p[i < np ? i : 0];
    }
  }
  double sums[3];
  dev::sum_partials_n<3>({part_s, part_x, part_r}, {gs, gx, gr}, sums, red);
  const double ss = sums[0], xx = sums[1], rr = sums[2];
  double beta = 0.0;
  if (k >= 0) {
    const double gold = gamma[k];
    beta = (*status >= 0 || !(gold > 0.0)) ? 0.0 : ss / gold;
  }
  double acc = 0.0;
  const int64_t n = np > m ? np : m;
#pragma unroll
  for (int u = 0; u < kPrefetch; ++u) {
    const int64_t i = i0 + u * stride;
    if (i < np) {
      const T t = (T)((double)sv[u] + (beta != 0.0 ? beta * (double)pv[u] : 0.0));
      p[i] = t;
      acc += (double)t * (double)t;
    }
    if (i < m) q[i] = (T)0;
  }
  for (int64_t i = i0 + kPrefetch * stride; i < n; i += stride) {
    if (i < np) {
      const T t = (T)((double)s[i] + (beta != 0.0 ? beta * (double)p[i] : 0.0));
      p[i] = t;
      acc += (double)t * (double)t;
    }
    if (i < m) q[i] = (T)0;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) {
    part_p[bid] = acc;
    if (bid == 0) {
      gamma[k + 1] = ss;
      if (hist) {
        hist[3 * (k + 1) + 0] = sqrt(rr);
        hist[3 * (k + 1) + 1] = sqrt(ss);
        hist[3 * (k + 1) + 2] = rr + lambda * xx;
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) init_r_kernel(T* __restrict__ r, const T* __restrict__ y, const T* __restrict__ q,
                                                        int64_t m, double* __restrict__ part_r, int* __restrict__ status,
                                                        double* __restrict__ alpha0) {
  init_r_body<T>(blockIdx.x, gridDim.x, r, y, q, m, part_r, status, alpha0);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) upd_r_kernel(T* __restrict__ r, const T* __restrict__ q, int64_t m,
                                                       const double* __restrict__ part_q, int gq,
                                                       const double* __restrict__ part_p, int gp, double lambda,
                                                       const double* __restrict__ gamma_k, double* __restrict__ alpha_k,
                                                       int* __restrict__ status, int k, double* __restrict__ part_r) {
  upd_r_body<T>(blockIdx.x, gridDim.x, r, q, m, part_q, gq, part_p, gp, lambda, gamma_k, alpha_k, status, k, part_r);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) dir_kernel(T* __restrict__ p, const T* __restrict__ s, int64_t np,
                                                     T* __restrict__ q, int64_t m,
                                                     const double* __restrict__ part_s, int gs,
                                                     const double* __restrict__ part_x, int gx,
                                                     const double* __restrict__ part_r, int gr, double lambda,
                                                     double* __restrict__ gamma, int k, const int* __restrict__ status,
                                                     double* __restrict__ hist, double* __restrict__ part_p) {
  dir_body<T>(blockIdx.x, gridDim.x, p, s, np, q, m, part_s, gs, part_x, gx, part_r, gr, lambda, gamma, k, status, hist,
              part_p);
}

// ------------------------------------------------------------------ batches
// Frame f's state: status[f], gamma and alpha at f * astride, history at
// f * hstride; vectors at the frame's packed offsets.

template <typename T>
__global__ void __launch_bounds__(kBlock) init_r_batched(const FrameDesc* __restrict__ B, int nf, T* __restrict__ r,
                                                         const T* __restrict__ y, const T* __restrict__ q,
                                                         double* __restrict__ part_r, int* __restrict__ status,
                                                         double* __restrict__ alpha, int astride) {
  const int g = blockIdx.x;
  const FrameDesc& F = B[find_frame<&FrameDesc::b_m>(B, nf, g)];
  const int64_t m = (int64_t)F.op.S * F.op.K;
  init_r_body<T>(g - F.b_m, F.n_m, r + F.yo, y + F.yo, q ? q + F.yo : nullptr, m, part_r + F.b_m, status + F.frame,
                 alpha + (size_t)F.frame * astride);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) upd_r_batched(const FrameDesc* __restrict__ B, int nf, T* __restrict__ r,
                                                        const T* __restrict__ q, const double* __restrict__ part_q,
                                                        const double* __restrict__ part_p, double lambda,
                                                        const double* __restrict__ gamma, double* __restrict__ alpha,
                                                        int astride, int* __restrict__ status, int k,
                                                        double* __restrict__ part_r) {
  const int g = blockIdx.x;
  const FrameDesc& F = B[find_frame<&FrameDesc::b_m>(B, nf, g)];
  const int64_t m = (int64_t)F.op.S * F.op.K;
  const size_t a0 = (size_t)F.frame * astride;
  upd_r_body<T>(g - F.b_m, F.n_m, r + F.yo, q + F.yo, m, part_q + F.s_fp, F.n_fp > 0 ? F.n_fp : 1, part_p + F.b_p,
                F.n_p, lambda, gamma + a0 + k, alpha + a0 + k + 1, status + F.frame, k, part_r + F.b_m);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) dir_batched(const FrameDesc* __restrict__ B, int nf, T* __restrict__ p,
                                                      const T* __restrict__ s, const double* __restrict__ part_s,
                                                      const double* __restrict__ part_x,
                                                      const double* __restrict__ part_r, double lambda,
                                                      double* __restrict__ gamma, int astride, int k,
                                                      const int* __restrict__ status, double* __restrict__ hist,
                                                      int hstride, double* __restrict__ part_p) {
  const int g = blockIdx.x;
  const FrameDesc& F = B[find_frame<&FrameDesc::b_p>(B, nf, g)];
  const int64_t np = (int64_t)F.op.nx * F.op.ny * F.op.nz;
  const int gs = F.n_bp > 0 ? F.n_bp : 1;
  dir_body<T>(g - F.b_p, F.n_p, p + F.xo, s + F.xo, np, (T*)nullptr, 0, part_s + F.s_bp, gs, part_x + F.s_bp, gs,
              part_r + F.b_m, F.n_m, lambda, gamma + (size_t)F.frame * astride, k, status + F.frame,
              hist ? hist + (size_t)F.frame * hstride : nullptr, part_p + F.b_p);
}

hipError_t launch_fill(pa_dtype dt, void* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int g = blas_grid(n);
  if (dt == PA_F32) fill_kernel<float><<<g, kBlock, 0, st>>>(static_cast<float*>(p), n);
  else fill_kernel<double><<<g, kBlock, 0, st>>>(static_cast<double*>(p), n);
  return hipGetLastError();
}

hipError_t launch_init_r(pa_dtype dt, void* r, const void* y, const void* q, int64_t m, double* part_r, int* status,
                         double* alpha0, hipStream_t st) {
  const int g = blas_grid(m);
  if (dt == PA_F32)
    init_r_kernel<float><<<g, kBlock, 0, st>>>(static_cast<float*>(r), static_cast<const float*>(y),
                                               static_cast<const float*>(q), m, part_r, status, alpha0);
  else
    init_r_kernel<double><<<g, kBlock, 0, st>>>(static_cast<double*>(r), static_cast<const double*>(y),
                                                static_cast<const double*>(q), m, part_r, status, alpha0);
  return hipGetLastError();
}

hipError_t launch_upd_r(pa_dtype dt, void* r, const void* q, int64_t m, const double* part_q, int gq, const double* part_p,
                        int gp, double lambda, const double* gamma_k, double* alpha_k, int* status, int k, double* part_r,
                        hipStream_t st) {
  const int g = blas_grid(m);
  if (dt == PA_F32)
    upd_r_kernel<float><<<g, kBlock, 0, st>>>(static_cast<float*>(r), static_cast<const float*>(q), m, part_q, gq, part_p,
                                              gp, lambda, gamma_k, alpha_k, status, k, part_r);
  else
    upd_r_kernel<double><<<g, kBlock, 0, st>>>(static_cast<double*>(r), static_cast<const double*>(q), m, part_q, gq,
                                               part_p, gp, lambda, gamma_k, alpha_k, status, k, part_r);
  return hipGetLastError();
}

hipError_t launch_dir(pa_dtype dt, void* p, const void* s, int64_t np, void* q, int64_t m, const double* part_s, int gs,
                      const double* part_x, int gx, const double* part_r, int gr, double lambda, double* gamma, int k,
                      const int* status, double* hist, double* part_p, hipStream_t st) {
  const int g = blas_grid(np);
  if (dt == PA_F32)
    dir_kernel<float><<<g, kBlock, 0, st>>>(static_cast<float*>(p), static_cast<const float*>(s), np,
                                            static_cast<float*>(q), m, part_s, gs, part_x, gx, part_r, gr, lambda, gamma,
                                            k, status, hist, part_p);
  else
    dir_kernel<double><<<g, kBlock, 0, st>>>(static_cast<double*>(p), static_cast<const double*>(s), np,
                                             static_cast<double*>(q), m, part_s, gs, part_x, gx, part_r, gr, lambda,
                                             gamma, k, status, hist, part_p);
  return hipGetLastError();
}

hipError_t launch_init_r_batched(const BatchLaunch& L, void* r, const void* y, const void* q, double* part_r,
                                 int* status, double* alpha, int astride, hipStream_t st) {
  if (L.dtype == PA_F32)
    init_r_batched<float><<<L.m_grid, kBlock, 0, st>>>(L.table, L.nf, static_cast<float*>(r),
                                                       static_cast<const float*>(y), static_cast<const float*>(q),
                                                       part_r, status, alpha, astride);
  else
    init_r_batched<double><<<L.m_grid, kBlock, 0, st>>>(L.table, L.nf, static_cast<double*>(r),
                                                        static_cast<const double*>(y), static_cast<const double*>(q),
                                                        part_r, status, alpha, astride);
  return hipGetLastError();
}

hipError_t launch_upd_r_batched(const BatchLaunch& L, void* r, const void* q, const double* part_q,
                                const double* part_p, double lambda, const double* gamma, double* alpha, int astride,
                                int* status, int k, double* part_r, hipStream_t st) {
  if (L.dtype == PA_F32)
    upd_r_batched<float><<<L.m_grid, kBlock, 0, st>>>(L.table, L.nf, static_cast<float*>(r),
                                                      static_cast<const float*>(q), part_q, part_p, lambda, gamma,
                                                      alpha, astride, status, k, part_r);
  else
    upd_r_batched<double><<<L.m_grid, kBlock, 0, st>>>(L.table, L.nf, static_cast<double*>(r),
                                                       static_cast<const double*>(q), part_q, part_p, lambda, gamma,
                                                       alpha, astride, status, k, part_r);
  return hipGetLastError();
}

hipError_t launch_dir_batched(const BatchLaunch& L, void* p, const void* s, const double* part_s, const double* part_x,
                              const double* part_r, double lambda, double* gamma, int astride, int k,
                              const int* status, double* hist, int hstride, double* part_p, hipStream_t st) {
  if (L.dtype == PA_F32)
    dir_batched<float><<<L.p_grid, kBlock, 0, st>>>(L.table, L.nf, static_cast<float*>(p),
                                                    static_cast<const float*>(s), part_s, part_x, part_r, lambda,
                                                    gamma, astride, k, status, hist, hstride, part_p);
  else
    dir_batched<double><<<L.p_grid, kBlock, 0, st>>>(L.table, L.nf, static_cast<double*>(p),
                                                     static_cast<const double*>(s), part_s, part_x, part_r, lambda,
                                                     gamma, astride, k, status, hist, hstride, part_p);
  return hipGetLastError();
}

// ------------------------------------------------------ gradient iteration
// Landweber steps and the power iteration that estimates their step size.

template <typename T>
__global__ void __launch_bounds__(kBlock) fill_value_kernel(T* __restrict__ p, int64_t n, double v) {
  const T t = (T)v;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = t;
}

// partial sums of ||v||^2
template <typename T>
__global__ void __launch_bounds__(kBlock) norm2_kernel(const T* __restrict__ v, int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double t = (double)v[i];
    acc += t * t;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// sigma2 = ||w|| (w = A^T A v with ||v|| = 1), v = w / sigma2.
template <typename T>
__global__ void __launch_bounds__(kBlock) pw_scale_kernel(T* __restrict__ v, const T* __restrict__ w, int64_t n,
                                                          const double* __restrict__ part, int gp,
                                                          double* __restrict__ sigma2) {
  __shared__ double red[4];
  const double nw = sqrt(sum_partials(part, gp, red));
  const double inv = nw > 0.0 ? 1.0 / nw : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    v[i] = (T)((double)w[i] * inv);
  if (blockIdx.x == 0 && threadIdx.x == 0) *sigma2 = nw;
}

// omega = 1 / (sigma2 + lambda), or the caller's omega when it is > 0.
__global__ void pw_omega_kernel(const double* __restrict__ sigma2, double lambda, double given,
                                double* __restrict__ omega) {
  if (threadIdx.x == 0) {
    const double d = *sigma2 + lambda;
    *omega = given > 0.0 ? given : (d > 0.0 ? 1.0 / d : 0.0);
  }
}

// hist[k] = ||r_k||^2 + lambda ||x_k||^2 from the partials; then x += omega s.
template <typename T>
__global__ void __launch_bounds__(kBlock) lw_step_kernel(T* __restrict__ x, const T* __restrict__ s, int64_t np,
                                                         const double* __restrict__ part_r, int gr,
                                                         const double* __restrict__ part_x, int gx, double lambda,
                                                         const double* __restrict__ omega, double* __restrict__ hist,
                                                         int k) {
  __shared__ double red[4];
  const double rr = sum_partials(part_r, gr, red);
  const double xx = sum_partials(part_x, gx, red);
  const double w = *omega;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < np; i += (int64_t)gridDim.x * kBlock)
    x[i] = (T)((double)x[i] + w * (double)s[i]);
  if (hist && blockIdx.x == 0 && threadIdx.x == 0) hist[k] = rr + lambda * xx;
}

__global__ void lw_final_kernel(const double* __restrict__ part_r, int gr, const double* __restrict__ part_x, int gx,
                                double lambda, double* __restrict__ hist, int k) {
  __shared__ double red[4];
  const double rr = sum_partials(part_r, gr, red);
  const double xx = sum_partials(part_x, gx, red);
  if (hist && threadIdx.x == 0) hist[k] = rr + lambda * xx;
}

hipError_t launch_fill_value(pa_dtype dt, void* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int g = blas_grid(n);
  if (dt == PA_F32) fill_value_kernel<float><<<g, kBlock, 0, st>>>(static_cast<float*>(p), n, v);
  else fill_value_kernel<double><<<g, kBlock, 0, st>>>(static_cast<double*>(p), n, v);
  return hipGetLastError();
}

hipError_t launch_norm2(pa_dtype dt, const void* v, int64_t n, double* part, hipStream_t st) {
  const int g = blas_grid(n);
  if (dt == PA_F32) norm2_kernel<float><<<g, kBlock, 0, st>>>(static_cast<const float*>(v), n, part);
  else norm2_kernel<double><<<g, kBlock, 0, st>>>(static_cast<const double*>(v), n, part);
  return hipGetLastError();
}

hipError_t launch_pw_scale(pa_dtype dt, void* v, const void* w, int64_t n, const double* part, double* sigma2,
                           hipStream_t st) {
  const int g = blas_grid(n);
  if (dt == PA_F32)
    pw_scale_kernel<float><<<g, kBlock, 0, st>>>(static_cast<float*>(v), static_cast<const float*>(w), n, part, g,
                                                 sigma2);
  else
    pw_scale_kernel<double><<<g, kBlock, 0, st>>>(static_cast<double*>(v), static_cast<const double*>(w), n, part, g,
                                                  sigma2);
  return hipGetLastError();
}

hipError_t launch_pw_omega(const double* sigma2, double lambda, double given, double* omega, hipStream_t st) {
  pw_omega_kernel<<<1, 64, 0, st>>>(sigma2, lambda, given, omega);
  return hipGetLastError();
}

hipError_t launch_lw_step(pa_dtype dt, void* x, const void* s, int64_t np, const double* part_r, int gr,
                          const double* part_x, int gx, double lambda, const double* omega, double* hist, int k,
                          hipStream_t st) {
  const int g = blas_grid(np);
  if (dt == PA_F32)
    lw_step_kernel<float><<<g, kBlock, 0, st>>>(static_cast<float*>(x), static_cast<const float*>(s), np, part_r, gr,
                                                part_x, gx, lambda, omega, hist, k);
  else
    lw_step_kernel<double><<<g, kBlock, 0, st>>>(static_cast<double*>(x), static_cast<const double*>(s), np, part_r,
                                                 gr, part_x, gx, lambda, omega, hist, k);
  return hipGetLastError();
}

hipError_t launch_lw_final(const double* part_r, int gr, const double* part_x, int gx, double lambda, double* hist,
                           int k, hipStream_t st) {
  lw_final_kernel<<<1, kBlock, 0, st>>>(part_r, gr, part_x, gx, lambda, hist, k);
  return hipGetLastError();
}


// ------------------------------------------------ proximal gradient (FISTA)
// Objective ||A x - y||^2 + lambda ||x||^2 + beta TV_eps(x) + alpha ||x||_1
// (Eq. 8 with identity transforms).  TV_eps(z) = sum_p m_p with
// m_p = sqrt(dx_p^2 + dy_p^2 + eps^2) over forward differences of the 2D
// image (zero past the last column and row); its gradient at p collects
// dx/m of the pixel to the left, dy/m of the pixel above and -(dx + dy)/m of
// p itself.  Every per-pixel value is formed in FP64 from the stored z.

// Forward differences at a pixel of value zp from its right (zr) and lower
// (zd) neighbours, zero across the image's far edges, and their m.
__device__ __forceinline__ double tv_m(double zp, double zr, double zd, bool has_r, bool has_d, double eps2,
                                       double* dx, double* dy) {
  *dx = has_r ? zr - zp : 0.0;
  *dy = has_d ? zd - zp : 0.0;
  return sqrt(*dx * *dx + *dy * *dy + eps2);
}

__device__ __forceinline__ double shrink(double v, double tau, int nonneg) {
  if (nonneg) return v > tau ? v - tau : 0.0;
  return v > tau ? v - tau : (v < -tau ? v + tau : 0.0);
}

// One proximal step at the extrapolated point z, whose A^T (y - A z) - lambda z
// is s:  x_new = shrink(z + omega (s - beta/2 dTV(z)), omega alpha / 2),
// z_next = x_new + mu (x_new - x_old).  x is updated in place; z_next is a
// different buffer from z (neighbours of z are read).  Partials: TV(z) and
// ||z||_1 (the objective at z).  beta == 0 skips the TV term (any ndim).
template <typename T>
__global__ void __launch_bounds__(kBlock) fista_step_kernel(const T* __restrict__ z, const T* __restrict__ s,
                                                            T* __restrict__ x, T* __restrict__ zn, int nx, int ny,
                                                            int64_t np, double beta, double eps, double alpha,
                                                            const double* __restrict__ omega, double mu, int nonneg,
                                                            double* __restrict__ part_tv, double* __restrict__ part_l1) {
  __shared__ double red[4];
  const double w = *omega;
  const double tau = w * alpha * 0.5;
  const double eps2 = eps * eps;
  double acc_tv = 0.0, acc_l1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < np; i += (int64_t)gridDim.x * kBlock) {
    // every value this pixel needs is loaded up front (a neighbour across an
    // edge reads the pixel itself and is not used), so the loads go out
    // back to back
    const T zi_t = z[i], si_t = s[i], xi_t = x[i];
    const int ix = (int)(i % nx), iy = (int)(i / nx);
    const bool r = ix + 1 < nx, d = iy + 1 < ny, l = ix > 0, u = iy > 0;
    T zr = zi_t, zd = zi_t, zl = zi_t, zld = zi_t, zu = zi_t, zur = zi_t;
    if (beta != 0.0) {
      zr = z[r ? i + 1 : i];
      zd = z[d ? i + nx : i];
      zl = z[l ? i - 1 : i];
      zld = z[l && d ? i - 1 + nx : i];
      zu = z[u ? i - nx : i];
      zur = z[u && r ? i - nx + 1 : i];
    }
    const double zi = (double)zi_t;
    acc_l1 += fabs(zi);
    double gtv = 0.0;
    if (beta != 0.0) {
      double dx, dy, ex, ey;
      const double m = tv_m(zi, (double)zr, (double)zd, r, d, eps2, &dx, &dy);
      acc_tv += m;
      gtv = -(dx + dy) / m;
      if (l) {   // the left neighbour's differences (its right neighbour is this pixel)
        const double ml = tv_m((double)zl, zi, (double)zld, true, d, eps2, &ex, &ey);
        gtv += ex / ml;
      }
      if (u) {   // the upper neighbour's (its lower neighbour is this pixel)
        const double mu_ = tv_m((double)zu, (double)zur, zi, r, true, eps2, &ex, &ey);
        gtv += ey / mu_;
      }
    }
    const double v = zi + w * ((double)si_t - 0.5 * beta * gtv);
    const T xn = (T)shrink(v, tau, nonneg);
    const double xd = (double)xn;
    zn[i] = (T)(xd + mu * (xd - (double)xi_t));
    x[i] = xn;
  }
  acc_tv = block_sum(acc_tv, red);
  acc_l1 = block_sum(acc_l1, red);
  if (threadIdx.x == 0) {
    part_tv[blockIdx.x] = acc_tv;
    part_l1[blockIdx.x] = acc_l1;
  }
}

// Partials of ||v||^2, TV(v) (when beta != 0) and ||v||_1 (the objective at
// the final iterate).
template <typename T>
__global__ void __launch_bounds__(kBlock) fista_terms_kernel(const T* __restrict__ v, int nx, int ny, int64_t np,
                                                             double beta, double eps, double* __restrict__ part_n,
                                                             double* __restrict__ part_tv,
                                                             double* __restrict__ part_l1) {
  __shared__ double red[4];
  const double eps2 = eps * eps;
  double a2 = 0.0, atv = 0.0, a1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < np; i += (int64_t)gridDim.x * kBlock) {
    const T vi = v[i];
    const int ix = (int)(i % nx), iy = (int)(i / nx);
    const bool r = ix + 1 < nx, d = iy + 1 < ny;
    T vr = vi, vd = vi;
    if (beta != 0.0) {   // (loaded together; across an edge, the pixel itself)
      vr = v[r ? i + 1 : i];
      vd = v[d ? i + nx : i];
    }
    const double t = (double)vi;
    a2 += t * t;
    a1 += fabs(t);
    if (beta != 0.0) {
      double dx, dy;
      atv += tv_m(t, (double)vr, (double)vd, r, d, eps2, &dx, &dy);
    }
  }
  a2 = block_sum(a2, red);
  atv = block_sum(atv, red);
  a1 = block_sum(a1, red);
  if (threadIdx.x == 0) {
    part_n[blockIdx.x] = a2;
    part_tv[blockIdx.x] = atv;
    part_l1[blockIdx.x] = a1;
  }
}

// hist[k] = ||r||^2 + lambda ||v||^2 + beta TV(v) + alpha ||v||_1 from partials.
__global__ void fista_hist_kernel(const double* __restrict__ part_r, int gr, const double* __restrict__ part_n, int gn,
                                  const double* __restrict__ part_tv, const double* __restrict__ part_l1, int gp,
                                  double lambda, double beta, double alpha, double* __restrict__ hist, int k) {
  __shared__ double red[4];
  const double rr = sum_partials(part_r, gr, red);
  const double nn = sum_partials(part_n, gn, red);
  const double tv = beta != 0.0 ? sum_partials(part_tv, gp, red) : 0.0;
  const double l1 = sum_partials(part_l1, gp, red);
  if (threadIdx.x == 0) hist[k] = rr + lambda * nn + beta * tv + alpha * l1;
}

hipError_t launch_fista_step(pa_dtype dt, const void* z, const void* s, void* x, void* zn, int nx, int ny, int64_t np,
                             double beta, double eps, double alpha, const double* omega, double mu, int nonneg,
                             double* part_tv, double* part_l1, hipStream_t st) {
  const int g = blas_grid(np);
  if (dt == PA_F32)
    fista_step_kernel<float><<<g, kBlock, 0, st>>>(static_cast<const float*>(z), static_cast<const float*>(s),
                                                   static_cast<float*>(x), static_cast<float*>(zn), nx, ny, np, beta,
                                                   eps, alpha, omega, mu, nonneg, part_tv, part_l1);
  else
    fista_step_kernel<double><<<g, kBlock, 0, st>>>(static_cast<const double*>(z), static_cast<const double*>(s),
                                                    static_cast<double*>(x), static_cast<double*>(zn), nx, ny, np,
                                                    beta, eps, alpha, omega, mu, nonneg, part_tv, part_l1);
  return hipGetLastError();
}

hipError_t launch_fista_terms(pa_dtype dt, const void* v, int nx, int ny, int64_t np, double beta, double eps,
                              double* part_n, double* part_tv, double* part_l1, hipStream_t st) {
  const int g = blas_grid(np);
  if (dt == PA_F32)
    fista_terms_kernel<float><<<g, kBlock, 0, st>>>(static_cast<const float*>(v), nx, ny, np, beta, eps, part_n,
                                                    part_tv, part_l1);
  else
    fista_terms_kernel<double><<<g, kBlock, 0, st>>>(static_cast<const double*>(v), nx, ny, np, beta, eps, part_n,
                                                     part_tv, part_l1);
  return hipGetLastError();
}

hipError_t launch_fista_hist(const double* part_r, int gr, const double* part_n, int gn, const double* part_tv,
                             const double* part_l1, int gp, double lambda, double beta, double alpha, double* hist,
                             int k, hipStream_t st) {
  if (!hist) return hipSuccess;
  fista_hist_kernel<<<1, kBlock, 0, st>>>(part_r, gr, part_n, gn, part_tv, part_l1, gp, lambda, beta, alpha, hist, k);
  return hipGetLastError();
}

}  // namespace pa
