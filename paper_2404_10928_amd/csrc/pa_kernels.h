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

// The CGLS direction update carried by the partial-row forward operator
// (PA_F32): its pass 1 forms p_k = s_k + beta p_{k-1} while staging the
// image, beta = ||s_k||^2 / gamma[k - 1] (0 for k = 0 or once the solve has
// stopped), exactly as the separate direction kernel would; the work-groups
// of the first sensor chunk write p_k and the FP64 partial sums of ||p_k||^2
// (one per forward tile), and work-group 0 writes gamma[k] = ||s_k||^2 and
// history row k.
struct CgDirArgs {
  const float* s;         // s_k
  const float* p_old;     // p_{k-1} (for k = 0, any P readable floats: beta is 0)
  float* p_new;           // p_k
  const double* part_s;   // partial sums of ||s_k||^2 ...
  const double* part_x;   // ... of ||x_k||^2 ...
  const double* part_r;   // ... and of ||r_k||^2
  int gs, gx, gr;         // their counts
  double lambda;
  double* gamma;
  const int* status;
  double* hist;           // may be NULL
  double* part_p;         // n_atiles partial sums of ||p_k||^2
  int k;
};

hipError_t launch_fill(pa_dtype dt, void* p, int64_t n, hipStream_t st);
// x := A^T y (or the CGLS epilogue when cg != nullptr)
hipError_t launch_adjoint(const Plan& pl, const void* y, void* x, const CgArgs* cg, hipStream_t st);
// y := A x; when part_q is not NULL it receives the FP64 partial sums of
// ||y||^2 (max(plan.fp_grid, 1) of them, or plan.gather_grid through partial
// rows).  With plan.two_pass and a scratch of plan.fwd_scratch bytes the
// partial-row method runs; otherwise the sensor-major one.
hipError_t launch_forward(const Plan& pl, const void* x, void* y, double* part_q, void* scratch, hipStream_t st);
// q := A p_k through partial rows with the direction update above folded into
// pass 1 (x is not read: p_k is formed from dir.s and dir.p_old).  Only for
// plans whose forward runs through partial rows (two_pass, fwd_scratch > 0,
// fp2_grid > 0).
hipError_t launch_forward_cg(const Plan& pl, const CgDirArgs& dir, float* q, double* part_q, void* scratch,
                             hipStream_t st);
hipError_t launch_init_r(pa_dtype dt, void* r, const void* y, const void* q, int64_t m, double* part_r, int* status,
                         double* alpha0, hipStream_t st);
hipError_t launch_upd_r(pa_dtype dt, void* r, const void* q, int64_t m, const double* part_q, int gq, const double* part_p,
                        int gp, double lambda, const double* gamma_k, double* alpha_k, int* status, int k, double* part_r,
                        hipStream_t st);
hipError_t launch_dir(pa_dtype dt, void* p, const void* s, int64_t np, void* q, int64_t m, const double* part_s, int gs,
                      const double* part_x, int gx, const double* part_r, int gr, double lambda, double* gamma, int k,
                      const int* status, double* hist, double* part_p, hipStream_t st);

// Gradient (Landweber) iteration and its power-iteration step size.
hipError_t launch_fill_value(pa_dtype dt, void* p, int64_t n, double v, hipStream_t st);
hipError_t launch_norm2(pa_dtype dt, const void* v, int64_t n, double* part, hipStream_t st);  // blas_grid(n) partials
hipError_t launch_pw_scale(pa_dtype dt, void* v, const void* w, int64_t n, const double* part, double* sigma2,
                           hipStream_t st);
hipError_t launch_pw_omega(const double* sigma2, double lambda, double given, double* omega, hipStream_t st);
hipError_t launch_lw_step(pa_dtype dt, void* x, const void* s, int64_t np, const double* part_r, int gr,
                          const double* part_x, int gx, double lambda, const double* omega, double* hist, int k,
                          hipStream_t st);
hipError_t launch_lw_final(const double* part_r, int gr, const double* part_x, int gx, double lambda, double* hist,
                           int k, hipStream_t st);

// Proximal gradient (FISTA) on the l1 + TV objective: one step at the
// extrapolated point z, the objective's terms at a vector, and a history entry.
hipError_t launch_fista_step(pa_dtype dt, const void* z, const void* s, void* x, void* zn, int nx, int ny, int64_t np,
                             double beta, double eps, double alpha, const double* omega, double mu, int nonneg,
                             double* part_tv, double* part_l1, hipStream_t st);   // blas_grid(np) partials
hipError_t launch_fista_terms(pa_dtype dt, const void* v, int nx, int ny, int64_t np, double beta, double eps,
                              double* part_n, double* part_tv, double* part_l1, hipStream_t st);
hipError_t launch_fista_hist(const double* part_r, int gr, const double* part_n, int gn, const double* part_tv,
                             const double* part_l1, int gp, double lambda, double beta, double alpha, double* hist,
                             int k, hipStream_t st);

// ------------------------------------------------------------------ batches

// Index of the frame whose block range of one batched launch contains global
// block g (ranges are consecutive in table order; empty ranges are skipped
// because they share their start with the next frame).
template <int32_t FrameDesc::*BEG>
__device__ __forceinline__ int find_frame(const FrameDesc* __restrict__ B, int nf, int g) {
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (B[mid].*BEG <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// What a batched launch needs: the device frame table and the totals.
struct BatchLaunch {
  const FrameDesc* table;   // device, nf entries
  int nf;
  pa_dtype dtype;
  int ndim;
  bool frac;                // some frame has a fractional t0 / dt
  bool ffix;                // forward with fixed-point tile rows (FP32 delay arithmetic)
  int bp_grid, fp_grid, m_grid, p_grid;
  size_t bp_lds, fp_lds;
  int64_t P_total, M_total;
};

// CGLS epilogue of the batched adjoint: per-frame alpha at
// alpha[frame * astride + acol].
struct BatchCg {
  void* x;
  const void* p;
  const double* alpha;
  int astride, acol;
  double lambda;
  double* part_s;
  double* part_x;
};

hipError_t launch_adjoint_batched(const BatchLaunch& L, const void* y, void* x, const BatchCg* cg, hipStream_t st);
hipError_t launch_forward_batched(const BatchLaunch& L, const void* x, void* y, double* part_q, hipStream_t st);
hipError_t launch_init_r_batched(const BatchLaunch& L, void* r, const void* y, const void* q, double* part_r,
                                 int* status, double* alpha, int astride, hipStream_t st);
hipError_t launch_upd_r_batched(const BatchLaunch& L, void* r, const void* q, const double* part_q,
                                const double* part_p, double lambda, const double* gamma, double* alpha, int astride,
                                int* status, int k, double* part_r, hipStream_t st);
hipError_t launch_dir_batched(const BatchLaunch& L, void* p, const void* s, const double* part_s, const double* part_x,
                              const double* part_r, double lambda, double* gamma, int astride, int k,
                              const int* status, double* hist, int hstride, double* part_p, hipStream_t st);

}  // namespace pa
