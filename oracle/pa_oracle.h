/* FP64 CPU oracle for the photoacoustic time-domain operator and the
 * regularised least-squares solve around it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path.
 *
 * Operator (time-domain measurement matrix, Eq. 6, with the 1/R spreading of
 * the Green's function of Eq. 7 and a unit-peak linear "hat" standing for the
 * delta on the sample grid):
 *   R_ps   = max(|r_p - r_s|, r_min)
 *   tau_ps = (R_ps / c - t0) / dt                      (delay in samples)
 *   y[s,k] = sum_p x_p * (1/R_ps) * max(0, 1 - |k - tau_ps|),  k = 0..K-1
 * Adjoint: x[p] = sum_s sum_k (1/R_ps) * max(0, 1 - |k - tau_ps|) * y[s,k].
 * Layouts: x is [nz][ny][nx] (ix fastest), y is [S][K] (k fastest).
 * Pixel (ix,iy,iz) sits at center + (i - (n-1)/2) * h on each axis.
 * r_min == 0 selects h/2.
 */
#ifndef PA_ORACLE_H
#define PA_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t ndim;
  int32_t nx, ny, nz;
  double h;
  double center[3];
  int32_t n_sensors;
  const double* sensors;   /* host, [S][ndim] */
  int32_t n_samples;
  double dt, t0, c, r_min;
} or_geom;

/* y := A x (full, two-tap form). Returns 0 on success, -1 on bad geometry. */
int or_forward(const or_geom* g, const double* x, double* y, int threads);
/* x := A^T y */
int or_adjoint(const or_geom* g, const double* y, double* x, int threads);
/* one output of A evaluated straight from the hat definition (all pixels) */
double or_forward_at(const or_geom* g, const double* x, int32_t s, int32_t k);
/* one output of A^T evaluated straight from the hat definition (all samples) */
double or_adjoint_at(const or_geom* g, const double* y, int64_t p);
/* CGLS on min ||A x - y||^2 + lambda ||x||^2.
 * x: in = x0 (ignored when x0_zero), out = x_N.
 * hist (may be NULL): [iters+1][3] = (||r_k||, ||s_k||, F_k = ||r_k||^2 + lambda ||x_k||^2).
 * Returns the iteration at which CGLS stopped early (gamma == 0 or delta == 0),
 * or iters when it ran to completion; -1 on bad geometry. */
int or_cgls(const or_geom* g, const double* y, double* x, int iters, double lambda,
            int x0_zero, double* hist, int threads);
/* Landweber: x <- x + omega * (A^T (y - A x) - lambda x), x0 = 0.
 * hist (may be NULL): [iters+1] = F_k. Returns 0 / -1. */
int or_landweber(const or_geom* g, const double* y, double* x, int iters, double lambda,
                 double omega, double* hist, int threads);
/* Largest eigenvalue of A^T A by `iters` power-iteration steps from the
 * all-ones vector (see the source). */
double or_power_sigma2(const or_geom* g, int iters, int threads);

/* Isotropic smoothed total variation of one 2D image [ny][nx] (the TV term of
 * the paper's objective, Eq. 8): TV = sum_p sqrt(dx_p^2 + dy_p^2 + eps^2) with
 * forward differences, zero past the last column / row.  Returns TV and, if
 * grad is not NULL, writes dTV/dx. */
double or_tv2d(const double* x, int32_t nx, int32_t ny, double eps, double* grad);

/* FISTA on F(x) = ||A x - y||^2 + lambda ||x||^2 + beta TV_eps(x) + alpha ||x||_1
 * (the objective of Eq. 8 with identity transforms), x0 = 0, fixed step omega;
 * nonneg adds the constraint x >= 0.  hz[k] = F(z_k) (k < iters), hz[iters] =
 * F(x_iters); hx[k] = F(x_k); either may be NULL.  TV needs ndim 2.  Returns 0 / -1. */
int or_fista(const or_geom* g, const double* y, double* x, int iters, double lambda, double alpha,
             double beta, double eps, double omega, int nonneg, double* hz, double* hx, int threads);

/* Frequency-domain matrix of Eq. 7, K(s,n)_p = i c k_n exp(-i k_n R)/R with
 * k_n = 2 pi (f0 + n df) / c, n = 0..nf-1.  Y: complex [S][nf][2] (re, im).
 * Forward Y = K x (real x); adjoint x = Re(K^H Y).  Returns 0 / -1. */
int or_freq_forward(const or_geom* g, double f0, double df, int32_t nf, const double* x, double* Y,
                    int threads);
int or_freq_adjoint(const or_geom* g, double f0, double df, int32_t nf, const double* Y, double* x,
                    int threads);

#ifdef __cplusplus
}
#endif
#endif
