/* FP64 CPU oracle: plain loops, no blocking, no fusion.
 * TEST INFRASTRUCTURE ONLY -- see pa_oracle.h.  Never linked into the product.
 */
#include "pa_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int geom_ok(const or_geom* g) {
  if (!g) return 0;
  if (g->ndim != 2 && g->ndim != 3) return 0;
  if (g->nx < 0 || g->ny < 0 || g->nz < 0) return 0;
  if (g->ndim == 2 && g->nz != 1) return 0;
  if (g->n_sensors < 0 || g->n_samples < 0) return 0;
  if (!(g->h > 0) || !(g->dt > 0) || !(g->c > 0) || !(g->r_min >= 0)) return 0;
  if (g->n_sensors > 0 && !g->sensors) return 0;
  return 1;
}

static int64_t npix(const or_geom* g) { return (int64_t)g->nx * g->ny * g->nz; }

static double rmin_of(const or_geom* g) { return g->r_min > 0 ? g->r_min : 0.5 * g->h; }

/* pixel centre: center + (i - (n-1)/2) h on each axis */
static void pixel_pos(const or_geom* g, int64_t p, double r[3]) {
  int64_t ix = p % g->nx;
  int64_t iy = (p / g->nx) % g->ny;
  int64_t iz = p / ((int64_t)g->nx * g->ny);
  r[0] = g->center[0] + ((double)ix - 0.5 * (g->nx - 1)) * g->h;
  r[1] = g->center[1] + ((double)iy - 0.5 * (g->ny - 1)) * g->h;
  r[2] = g->center[2] + ((double)iz - 0.5 * (g->nz - 1)) * g->h;
}

/* distance R_ps (clamped) between pixel p and sensor s */
static double dist(const or_geom* g, int64_t p, int32_t s) {
  double r[3];
  pixel_pos(g, p, r);
  const double* q = g->sensors + (int64_t)s * g->ndim;
  double d2 = 0.0;
  for (int a = 0; a < g->ndim; ++a) d2 += (r[a] - q[a]) * (r[a] - q[a]);
  double R = sqrt(d2);
  double rm = rmin_of(g);
  return R > rm ? R : rm;
}

/* delay of an arrival in sample units */
static double delay(const or_geom* g, double R) { return (R / g->c - g->t0) / g->dt; }

static double hat(double u) {
  double a = 1.0 - fabs(u);
  return a > 0.0 ? a : 0.0;
}

static void set_threads(int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
}

int or_forward(const or_geom* g, const double* x, double* y, int threads) {
  if (!geom_ok(g)) return -1;
  const int32_t S = g->n_sensors, K = g->n_samples;
  const int64_t P = npix(g);
  set_threads(threads);
  /* each sensor row is owned by one thread: fixed summation order over p */
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t s = 0; s < S; ++s) {
    double* row = y + (int64_t)s * K;
    for (int32_t k = 0; k < K; ++k) row[k] = 0.0;
    for (int64_t p = 0; p < P; ++p) {
      double R = dist(g, p, s);
      double tau = delay(g, R);
      double k0d = floor(tau);
      double f = tau - k0d;
      double w = 1.0 / R;
      if (k0d >= 0.0 && k0d <= (double)(K - 1)) row[(int64_t)k0d] += w * (1.0 - f) * x[p];
      if (k0d + 1.0 >= 0.0 && k0d + 1.0 <= (double)(K - 1)) row[(int64_t)k0d + 1] += w * f * x[p];
    }
  }
  return 0;
}

int or_adjoint(const or_geom* g, const double* y, double* x, int threads) {
  if (!geom_ok(g)) return -1;
  const int32_t S = g->n_sensors, K = g->n_samples;
  const int64_t P = npix(g);
  set_threads(threads);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < P; ++p) {
    double acc = 0.0;
    for (int32_t s = 0; s < S; ++s) {
      const double* row = y + (int64_t)s * K;
      double R = dist(g, p, s);
      double tau = delay(g, R);
      double k0d = floor(tau);
      double f = tau - k0d;
      double w = 1.0 / R;
      if (k0d >= 0.0 && k0d <= (double)(K - 1)) acc += w * (1.0 - f) * row[(int64_t)k0d];
      if (k0d + 1.0 >= 0.0 && k0d + 1.0 <= (double)(K - 1)) acc += w * f * row[(int64_t)k0d + 1];
    }
    x[p] = acc;
  }
  return 0;
}

double or_forward_at(const or_geom* g, const double* x, int32_t s, int32_t k) {
  if (!geom_ok(g) || s < 0 || s >= g->n_sensors || k < 0 || k >= g->n_samples) return NAN;
  const int64_t P = npix(g);
  double acc = 0.0;
  for (int64_t p = 0; p < P; ++p) {
    double R = dist(g, p, s);
    acc += x[p] * hat((double)k - delay(g, R)) / R;
  }
  return acc;
}

double or_adjoint_at(const or_geom* g, const double* y, int64_t p) {
  if (!geom_ok(g) || p < 0 || p >= npix(g)) return NAN;
  double acc = 0.0;
  for (int32_t s = 0; s < g->n_sensors; ++s) {
    double R = dist(g, p, s);
    double tau = delay(g, R);
    for (int32_t k = 0; k < g->n_samples; ++k)
      acc += hat((double)k - tau) / R * y[(int64_t)s * g->n_samples + k];
  }
  return acc;
}

static double dot(const double* a, const double* b, int64_t n) {
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) acc += a[i] * b[i];
  return acc;
}

/* CGLS (Hestenes-Stiefel CG on the shifted normal equations, Bjorck's form):
 *   r = y - A x;  s = A^T r - lambda x;  p = s;  gamma = ||s||^2
 *   repeat: q = A p;  delta = ||q||^2 + lambda ||p||^2;  alpha = gamma / delta
 *           x += alpha p;  r -= alpha q;  s = A^T r - lambda x
 *           gamma' = ||s||^2;  beta = gamma' / gamma;  p = s + beta p
 * It minimises F(x) = ||A x - y||^2 + lambda ||x||^2; s = -grad F / 2. */
int or_cgls(const or_geom* g, const double* y, double* x, int iters, double lambda,
            int x0_zero, double* hist, int threads) {
  if (!geom_ok(g) || iters < 0 || !(lambda >= 0)) return -1;
  const int64_t P = npix(g);
  const int64_t M = (int64_t)g->n_sensors * g->n_samples;
  double* r = (double*)malloc(sizeof(double) * (M ? M : 1));
  double* q = (double*)malloc(sizeof(double) * (M ? M : 1));
  double* s = (double*)malloc(sizeof(double) * (P ? P : 1));
  double* p = (double*)malloc(sizeof(double) * (P ? P : 1));
  if (!r || !q || !s || !p) { free(r); free(q); free(s); free(p); return -1; }

  if (x0_zero) memset(x, 0, sizeof(double) * P);
  or_forward(g, x, q, threads);
  for (int64_t i = 0; i < M; ++i) r[i] = y[i] - q[i];
  or_adjoint(g, r, s, threads);
  for (int64_t i = 0; i < P; ++i) s[i] -= lambda * x[i];
  memcpy(p, s, sizeof(double) * P);
  double gamma = dot(s, s, P);
  if (hist) {
    double rr = dot(r, r, M);
    hist[0] = sqrt(rr);
    hist[1] = sqrt(gamma);
    hist[2] = rr + lambda * dot(x, x, P);
  }
  int stop = iters;
  for (int k = 0; k < iters; ++k) {
    or_forward(g, p, q, threads);
    double delta = dot(q, q, M) + lambda * dot(p, p, P);
    if (gamma == 0.0 || delta == 0.0 || !isfinite(delta) || !isfinite(gamma)) {
      stop = k;
      if (hist)
        for (int j = k + 1; j <= iters; ++j) memcpy(hist + 3 * j, hist + 3 * k, 3 * sizeof(double));
      break;
    }
    double alpha = gamma / delta;
    for (int64_t i = 0; i < P; ++i) x[i] += alpha * p[i];
    for (int64_t i = 0; i < M; ++i) r[i] -= alpha * q[i];
    or_adjoint(g, r, s, threads);
    for (int64_t i = 0; i < P; ++i) s[i] -= lambda * x[i];
    double gamma1 = dot(s, s, P);
    double beta = gamma1 / gamma;
    gamma = gamma1;
    for (int64_t i = 0; i < P; ++i) p[i] = s[i] + beta * p[i];
    if (hist) {
      double rr = dot(r, r, M);
      hist[3 * (k + 1) + 0] = sqrt(rr);
      hist[3 * (k + 1) + 1] = sqrt(gamma);
      hist[3 * (k + 1) + 2] = rr + lambda * dot(x, x, P);
    }
  }
  free(r); free(q); free(s); free(p);
  return stop;
}

/* Landweber / gradient iteration on the same objective with a fixed step:
 * x <- x + omega * (A^T (y - A x) - lambda x), i.e. x <- x - (omega/2) grad F. */
int or_landweber(const or_geom* g, const double* y, double* x, int iters, double lambda,
                 double omega, double* hist, int threads) {
  if (!geom_ok(g) || iters < 0 || !(lambda >= 0)) return -1;
  const int64_t P = npix(g);
  const int64_t M = (int64_t)g->n_sensors * g->n_samples;
  double* r = (double*)malloc(sizeof(double) * (M ? M : 1));
  double* s = (double*)malloc(sizeof(double) * (P ? P : 1));
  if (!r || !s) { free(r); free(s); return -1; }
  memset(x, 0, sizeof(double) * P);
  for (int k = 0; k <= iters; ++k) {
    or_forward(g, x, r, threads);
    for (int64_t i = 0; i < M; ++i) r[i] = y[i] - r[i];
    if (hist) hist[k] = dot(r, r, M) + lambda * dot(x, x, P);
    if (k == iters) break;
    or_adjoint(g, r, s, threads);
    for (int64_t i = 0; i < P; ++i) x[i] += omega * (s[i] - lambda * x[i]);
  }
  free(r); free(s);
  return 0;
}

/* Largest eigenvalue of A^T A by power iteration (the step-size estimate of
 * the gradient iteration): v_0 = (1, ..., 1) / sqrt(P); for each of `iters`
 * steps w = A^T A v, sigma2 = ||w||, v = w / ||w||.  Returns sigma2 after the
 * last step, 0 when A^T A v vanishes, or -1 on bad arguments. */
double or_power_sigma2(const or_geom* g, int iters, int threads) {
  if (!geom_ok(g) || iters < 1) return -1.0;
  const int64_t P = npix(g);
  const int64_t M = (int64_t)g->n_sensors * g->n_samples;
  if (P == 0 || M == 0) return 0.0;
  double* v = (double*)malloc(sizeof(double) * P);
  double* w = (double*)malloc(sizeof(double) * P);
  double* q = (double*)malloc(sizeof(double) * M);
  if (!v || !w || !q) { free(v); free(w); free(q); return -1.0; }
  for (int64_t i = 0; i < P; ++i) v[i] = 1.0 / sqrt((double)P);
  double sigma2 = 0.0;
  for (int it = 0; it < iters; ++it) {
    or_forward(g, v, q, threads);
    or_adjoint(g, q, w, threads);
    sigma2 = sqrt(dot(w, w, P));
    if (!(sigma2 > 0.0)) { sigma2 = 0.0; break; }
    for (int64_t i = 0; i < P; ++i) v[i] = w[i] / sigma2;
  }
  free(v); free(w); free(q);
  return sigma2;
}

/* TV_eps(x) = sum_p m_p, m_p = sqrt(dx_p^2 + dy_p^2 + eps^2),
 * dx_p = x[iy][ix+1] - x[iy][ix] (0 in the last column), dy_p likewise.
 * dTV/dx[q] collects, from every m_p whose differences contain x[q],
 * (d m_p / d dx_p) * (d dx_p / d x[q]) + (d m_p / d dy_p) * (d dy_p / d x[q]). */
double or_tv2d(const double* x, int32_t nx, int32_t ny, double eps, double* grad) {
  double tv = 0.0;
  if (grad)
    for (int64_t i = 0; i < (int64_t)nx * ny; ++i) grad[i] = 0.0;
  for (int32_t iy = 0; iy < ny; ++iy) {
    for (int32_t ix = 0; ix < nx; ++ix) {
      const int64_t p = (int64_t)iy * nx + ix;
      const double dx = ix + 1 < nx ? x[p + 1] - x[p] : 0.0;
      const double dy = iy + 1 < ny ? x[p + nx] - x[p] : 0.0;
      const double m = sqrt(dx * dx + dy * dy + eps * eps);
      tv += m;
      if (grad) {
        if (ix + 1 < nx) {
          grad[p + 1] += dx / m;
          grad[p] -= dx / m;
        }
        if (iy + 1 < ny) {
          grad[p + nx] += dy / m;
          grad[p] -= dy / m;
        }
      }
    }
  }
  return tv;
}

/* Soft threshold: the proximal map of tau * |v| (of tau * v + the indicator
 * of v >= 0 when nonneg). */
static double shrink(double v, double tau, int nonneg) {
  if (nonneg) return v > tau ? v - tau : 0.0;
  if (v > tau) return v - tau;
  if (v < -tau) return v + tau;
  return 0.0;
}

/* F(x) = ||A x - y||^2 + lambda ||x||^2 + beta TV_eps(x) + alpha ||x||_1,
 * with the TV term only when beta != 0.  r is scratch of S*K doubles. */
static double fista_objective(const or_geom* g, const double* y, const double* x, double lambda,
                              double alpha, double beta, double eps, double* r, int threads) {
  const int64_t P = npix(g);
  const int64_t M = (int64_t)g->n_sensors * g->n_samples;
  or_forward(g, x, r, threads);
  for (int64_t i = 0; i < M; ++i) r[i] -= y[i];
  double l1 = 0.0;
  for (int64_t i = 0; i < P; ++i) l1 += fabs(x[i]);
  double f = dot(r, r, M) + lambda * dot(x, x, P) + alpha * l1;
  if (beta != 0.0) f += beta * or_tv2d(x, g->nx, g->ny, eps, NULL);
  return f;
}

/* Accelerated proximal gradient (FISTA, Beck and Teboulle 2009) on the
 * objective of Eq. 8 with the sparsifying transforms taken as the identity,
 * plus a Tikhonov term:
 *   F(x) = ||A x - y||^2 + lambda ||x||^2 + beta TV_eps(x) + alpha ||x||_1.
 * The first three terms are smooth; half their gradient is
 *   G(z) = A^T (A z - y) + lambda z + (beta / 2) dTV_eps/dz.
 * From x_0 = z_0 = 0 and t_0 = 1, for k = 0 .. iters - 1:
 *   x_{k+1} = shrink(z_k - omega G(z_k), omega alpha / 2)
 *   t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
 *   z_{k+1} = x_{k+1} + ((t_k - 1) / t_{k+1}) (x_{k+1} - x_k)
 * (shrink keeps x >= 0 as well when nonneg).  omega is the step, 1 / L for
 * L = sigma2 + lambda + 4 beta / eps the Lipschitz constant of G.
 * hz (may be NULL): [iters + 1], hz[k] = F(z_k) for k < iters, hz[iters] = F(x_iters).
 * hx (may be NULL): [iters + 1], hx[k] = F(x_k).
 * The TV term needs a 2D image (ndim 2); returns -1 otherwise when beta != 0. */
int or_fista(const or_geom* g, const double* y, double* x, int iters, double lambda, double alpha,
             double beta, double eps, double omega, int nonneg, double* hz, double* hx, int threads) {
  if (!geom_ok(g) || iters < 0 || !(lambda >= 0) || !(alpha >= 0) || !(beta >= 0) || !(omega > 0)) return -1;
  if (beta != 0.0 && (g->ndim != 2 || !(eps > 0))) return -1;
  const int64_t P = npix(g);
  const int64_t M = (int64_t)g->n_sensors * g->n_samples;
  double* r = (double*)malloc(sizeof(double) * (M ? M : 1));
  double* z = (double*)malloc(sizeof(double) * (P ? P : 1));
  double* grad = (double*)malloc(sizeof(double) * (P ? P : 1));
  double* tvg = (double*)malloc(sizeof(double) * (P ? P : 1));
  double* xn = (double*)malloc(sizeof(double) * (P ? P : 1));
  if (!r || !z || !grad || !tvg || !xn) { free(r); free(z); free(grad); free(tvg); free(xn); return -1; }
  memset(x, 0, sizeof(double) * P);
  memset(z, 0, sizeof(double) * P);
  double t = 1.0;
  const double tau = omega * alpha / 2.0;
  if (hx) hx[0] = fista_objective(g, y, x, lambda, alpha, beta, eps, r, threads);
  for (int k = 0; k < iters; ++k) {
    if (hz) hz[k] = fista_objective(g, y, z, lambda, alpha, beta, eps, r, threads);
    /* G(z) */
    or_forward(g, z, r, threads);
    for (int64_t i = 0; i < M; ++i) r[i] -= y[i];
    or_adjoint(g, r, grad, threads);
    for (int64_t i = 0; i < P; ++i) grad[i] += lambda * z[i];
    if (beta != 0.0) {
      or_tv2d(z, g->nx, g->ny, eps, tvg);
      for (int64_t i = 0; i < P; ++i) grad[i] += 0.5 * beta * tvg[i];
    }
    for (int64_t i = 0; i < P; ++i) xn[i] = shrink(z[i] - omega * grad[i], tau, nonneg);
    const double t1 = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
    const double mu = (t - 1.0) / t1;
    for (int64_t i = 0; i < P; ++i) {
      z[i] = xn[i] + mu * (xn[i] - x[i]);
      x[i] = xn[i];
    }
    t = t1;
    if (hx) hx[k + 1] = fista_objective(g, y, x, lambda, alpha, beta, eps, r, threads);
  }
  if (hz) hz[iters] = hx ? hx[iters] : fista_objective(g, y, x, lambda, alpha, beta, eps, r, threads);
  free(r); free(z); free(grad); free(tvg); free(xn);
  return 0;
}

#define OR_TWO_PI 6.283185307179586476925286766559

/* Frequency-domain measurement matrix (Eq. 7):
 *   K(s, n)_p = i c k_n exp(-i k_n R_ps) / R_ps,   k_n = 2 pi f_n / c,
 *   f_n = f0 + n df, n = 0 .. nf-1,
 * so with c k_n = 2 pi f_n and e^{-i phi} = cos(phi) - i sin(phi):
 *   Re K = 2 pi f_n sin(k_n R) / R,   Im K = 2 pi f_n cos(k_n R) / R.
 * Y is complex, stored interleaved [S][nf][2] (re, im).  The time-domain
 * fields dt, t0 and n_samples of the geometry are not used.
 * or_freq_forward: Y = K x for a real image x.
 * or_freq_adjoint: x = Re(K^H Y), the adjoint for the real inner product
 *   <Y, Z> = sum Re(Y) Re(Z) + Im(Y) Im(Z). */
int or_freq_forward(const or_geom* g, double f0, double df, int32_t nf, const double* x, double* Y,
                    int threads) {
  if (!geom_ok(g) || nf < 0) return -1;
  const int32_t S = g->n_sensors;
  const int64_t P = npix(g);
  set_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t s = 0; s < S; ++s) {
    for (int32_t n = 0; n < nf; ++n) {
      const double fn = f0 + n * df;
      const double kn = OR_TWO_PI * fn / g->c;
      double re = 0.0, im = 0.0;
      for (int64_t p = 0; p < P; ++p) {
        const double R = dist(g, p, s);
        re += x[p] * OR_TWO_PI * fn * sin(kn * R) / R;
        im += x[p] * OR_TWO_PI * fn * cos(kn * R) / R;
      }
      Y[((int64_t)s * nf + n) * 2 + 0] = re;
      Y[((int64_t)s * nf + n) * 2 + 1] = im;
    }
  }
  return 0;
}

int or_freq_adjoint(const or_geom* g, double f0, double df, int32_t nf, const double* Y, double* x,
                    int threads) {
  if (!geom_ok(g) || nf < 0) return -1;
  const int32_t S = g->n_sensors;
  const int64_t P = npix(g);
  set_threads(threads);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < P; ++p) {
    double acc = 0.0;
    for (int32_t s = 0; s < S; ++s) {
      const double R = dist(g, p, s);
      for (int32_t n = 0; n < nf; ++n) {
        const double fn = f0 + n * df;
        const double kn = OR_TWO_PI * fn / g->c;
        const double kre = OR_TWO_PI * fn * sin(kn * R) / R;
        const double kim = OR_TWO_PI * fn * cos(kn * R) / R;
        acc += kre * Y[((int64_t)s * nf + n) * 2 + 0] + kim * Y[((int64_t)s * nf + n) * 2 + 1];
      }
    }
    x[p] = acc;
  }
  return 0;
}
