// Frequency-domain measurement matrix of Eq. 7 and its adjoint, matrix-free:
//   K(s, n)_p = i c k_n exp(-i k_n R_ps) / R_ps,  k_n = 2 pi f_n / c,
//   f_n = f0 + n df  (n = 0 .. nf-1),
// so  Re K = 2 pi f_n sin(2 pi f_n R / c) / R  and  Im K = 2 pi f_n cos(2 pi f_n R / c) / R.
//
// The phase is kept in cycles, f_n R / c = a + n b with a = f0 R / c and
// b = df R / c formed in FP64 per (pixel, sensor); a + n b is reduced to
// [-1/2, 1/2] in FP64 before the sine and cosine, so the phase error does not
// grow with the number of cycles (tens to thousands at ultrasound
// frequencies).  Sums are FP64.  Both products run in two passes: partial
// sums per work-group into a caller-owned workspace, then a fixed-order
// reduction, so results are reproducible run to run.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pa_freq.h"

namespace pa {
namespace {

constexpr int kT = 256;              // threads per work-group
constexpr int64_t kTargetBlocks = 4096;  // work-groups per launch the chunking aims for
constexpr double kTwoPi = 6.283185307179586476925286766559;

struct FreqGeom {
  int32_t ndim, nx, ny, nz, S, nf;
  int64_t P;
  double h, cx, cy, cz, c, rmin, f0, df;
  const double* sensors;   // device [S][ndim], metres
};

__device__ __forceinline__ double pixel_dist(const FreqGeom& g, int64_t p, int s) {
  const int ix = (int)(p % g.nx);
  const int64_t q = p / g.nx;
  const int iy = (int)(q % g.ny);
  const int iz = (int)(q / g.ny);
  const double* sp = g.sensors + (int64_t)s * g.ndim;
  const double dx = g.cx + ((double)ix - 0.5 * (g.nx - 1)) * g.h - sp[0];
  const double dy = g.cy + ((double)iy - 0.5 * (g.ny - 1)) * g.h - sp[1];
  double r2 = dx * dx + dy * dy;
  if (g.ndim == 3) {
    const double dz = g.cz + ((double)iz - 0.5 * (g.nz - 1)) * g.h - sp[2];
    r2 += dz * dz;
  }
  return fmax(sqrt(r2), g.rmin);
}

// sin and cos of 2 pi cyc for a phase in cycles.  FP32: the hardware sine and
// cosine take their argument in revolutions, so the reduced phase feeds them
// directly (|r| <= 1/2, well inside their domain).
__device__ __forceinline__ void sincos_cycles(double cyc, float* s, float* c) {
  const float r = (float)(cyc - rint(cyc));   // [-1/2, 1/2]; the subtraction is exact
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void sincos_cycles(double cyc, double* s, double* c) {
  const double r = cyc - rint(cyc);
  sincospi(2.0 * r, s, c);
}

// Forward, pass 1: work-group (sensor s, block of kT frequencies, chunk of
// `chunk` pixels); thread t owns frequency n = fb * kT + t.  Each round
// stages kT pixels' (a, b, x/R) in LDS, one per thread, then every thread
// runs over them.  part[(pc * S + s) * nf + n] = (sum x sin / R, sum x cos / R).
template <typename T>
__global__ void __launch_bounds__(kT) freq_fwd_kernel(FreqGeom g, const T* __restrict__ x, double2* __restrict__ part,
                                                      int nfb, int64_t chunk) {
  __shared__ double sa[kT], sb[kT];
  __shared__ T sw[kT];
  const int s = blockIdx.x % g.S;
  const int fb = (blockIdx.x / g.S) % nfb;
  const int pc = blockIdx.x / (g.S * nfb);
  const int n = fb * kT + threadIdx.x;
  const double dn = (double)n;
  const int64_t p0 = (int64_t)pc * chunk;
  const int64_t p1 = p0 + chunk < g.P ? p0 + chunk : g.P;
  double re = 0.0, im = 0.0;
  for (int64_t pb = p0; pb < p1; pb += kT) {
    const int64_t p = pb + threadIdx.x;
    __syncthreads();
    if (p < p1) {
      const double R = pixel_dist(g, p, s);
      const double t = R / g.c;
      sa[threadIdx.x] = g.f0 * t;
      sb[threadIdx.x] = g.df * t;
      sw[threadIdx.x] = (T)((double)x[p] / R);
    }
    __syncthreads();
    const int cnt = (int)(p1 - pb < kT ? p1 - pb : kT);
    for (int j = 0; j < cnt; ++j) {
      T sn, cs;
      sincos_cycles(fma(dn, sb[j], sa[j]), &sn, &cs);
      const double w = (double)sw[j];
      re = fma(w, (double)sn, re);
      im = fma(w, (double)cs, im);
    }
  }
  if (n < g.nf) part[((int64_t)pc * g.S + s) * g.nf + n] = make_double2(re, im);
}

// Forward, pass 2: Y[s][n] = 2 pi f_n * sum over pixel chunks (chunk order).
template <typename T>
__global__ void __launch_bounds__(kT) freq_fwd_reduce_kernel(FreqGeom g, const double2* __restrict__ part,
                                                             int nchunks, T* __restrict__ Y) {
  const int64_t m = (int64_t)g.S * g.nf;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT) {
    double re = 0.0, im = 0.0;
    for (int c = 0; c < nchunks; ++c) {
      const double2 v = part[(int64_t)c * m + i];
      re += v.x;
      im += v.y;
    }
    const double sc = kTwoPi * (g.f0 + (double)(i % g.nf) * g.df);
    Y[2 * i] = (T)(sc * re);
    Y[2 * i + 1] = (T)(sc * im);
  }
}

// Adjoint, pass 1: work-group (block of kT pixels, chunk of `sens` sensors);
// thread t owns pixel p.  For each sensor the frequency samples
// 2 pi f_n Y[s][n] are staged in LDS kT at a time; the phase a + n b steps by
// b in FP64.  part[sc * P + p] = sum over the chunk's sensors and all n of
// 2 pi f_n (Re Y sin + Im Y cos) / R.
template <typename T>
__global__ void __launch_bounds__(kT) freq_adj_kernel(FreqGeom g, const T* __restrict__ Y, double* __restrict__ part,
                                                      int npb, int sens) {
  __shared__ T yr[kT], yi[kT];
  const int pb = blockIdx.x % npb;
  const int sc = blockIdx.x / npb;
  const int64_t p = (int64_t)pb * kT + threadIdx.x;
  const bool live = p < g.P;
  const int s0 = sc * sens;
  const int s1 = s0 + sens < g.S ? s0 + sens : g.S;
  double acc = 0.0;
  for (int s = s0; s < s1; ++s) {
    double a = 0.0, b = 0.0, w = 0.0;
    if (live) {
      const double R = pixel_dist(g, p, s);
      const double t = R / g.c;
      a = g.f0 * t;
      b = g.df * t;
      w = 1.0 / R;
    }
    double sum = 0.0;
    for (int nb = 0; nb < g.nf; nb += kT) {
      const int n = nb + threadIdx.x;
      __syncthreads();
      if (n < g.nf) {
        const double sc2 = kTwoPi * (g.f0 + (double)n * g.df);
        const int64_t i = (int64_t)s * g.nf + n;
        yr[threadIdx.x] = (T)(sc2 * (double)Y[2 * i]);
        yi[threadIdx.x] = (T)(sc2 * (double)Y[2 * i + 1]);
      }
      __syncthreads();
      const int cnt = g.nf - nb < kT ? g.nf - nb : kT;
      if (live) {
        // phase of frequency nb, then one FP64 step of b per frequency
        double cyc = fma((double)nb, b, a);
        for (int j = 0; j < cnt; ++j) {
          T sn, cs;
          sincos_cycles(cyc, &sn, &cs);
          sum = fma((double)yr[j], (double)sn, fma((double)yi[j], (double)cs, sum));
          cyc += b;
        }
      }
    }
    acc += w * sum;
  }
  if (live) part[(int64_t)sc * g.P + p] = acc;
}

// Adjoint, pass 2: x[p] = sum over sensor chunks (chunk order).
template <typename T>
__global__ void __launch_bounds__(kT) freq_adj_reduce_kernel(const double* __restrict__ part, int nchunks, int64_t P,
                                                             T* __restrict__ x) {
  for (int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x; p < P; p += (int64_t)gridDim.x * kT) {
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * P + p];
    x[p] = (T)s;
  }
}

template <typename T>
__global__ void __launch_bounds__(kT) freq_zero_kernel(T* __restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) a[i] = (T)0;
}

int grid_for(int64_t n) {
  const int64_t g = (n + kT - 1) / kT;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

FreqGeom freq_geom(const pa_geometry* g, double f0, double df, int32_t nf) {
  FreqGeom d;
  d.ndim = g->ndim;
  d.nx = g->nx;
  d.ny = g->ny;
  d.nz = g->ndim == 3 ? g->nz : 1;
  d.S = g->n_sensors;
  d.nf = nf;
  d.P = (int64_t)d.nx * d.ny * d.nz;
  d.h = g->h;
  d.cx = g->center[0];
  d.cy = g->center[1];
  d.cz = g->center[2];
  d.c = g->c;
  d.rmin = g->r_min > 0.0 ? g->r_min : 0.5 * g->h;
  d.f0 = f0;
  d.df = df;
  d.sensors = g->sensors;
  return d;
}

}  // namespace

FreqShape freq_shape(int64_t P, int32_t S, int32_t nf) {
  FreqShape f;
  f.fwd_fblocks = (nf + kT - 1) / kT;
  // forward: pixel chunks (multiples of kT pixels) so that S * fblocks * chunks ~ kTargetBlocks
  const int64_t pblk = (P + kT - 1) / kT;
  const int64_t sf = (int64_t)(S > 0 ? S : 1) * (f.fwd_fblocks > 0 ? f.fwd_fblocks : 1);
  int64_t want = (kTargetBlocks + sf - 1) / sf;
  if (want > pblk) want = pblk;
  if (want < 1) want = 1;
  f.fwd_chunk_px = ((pblk + want - 1) / want) * kT;
  f.fwd_chunks = (int)((P + f.fwd_chunk_px - 1) / f.fwd_chunk_px);
  if (f.fwd_chunks < 1) f.fwd_chunks = 1;
  // adjoint: sensor chunks so that pixel blocks * chunks ~ kTargetBlocks
  f.adj_pblocks = (int)(pblk > 0 ? pblk : 1);
  int64_t nsc = (kTargetBlocks + f.adj_pblocks - 1) / f.adj_pblocks;
  if (nsc > S) nsc = S;
  if (nsc < 1) nsc = 1;
  f.adj_sens = (int)((S + nsc - 1) / nsc);
  if (f.adj_sens < 1) f.adj_sens = 1;
  f.adj_chunks = (S + f.adj_sens - 1) / f.adj_sens;
  if (f.adj_chunks < 1) f.adj_chunks = 1;
  const size_t fwd = sizeof(double) * 2 * (size_t)f.fwd_chunks * (size_t)S * (size_t)nf;
  const size_t adj = sizeof(double) * (size_t)f.adj_chunks * (size_t)P;
  f.workspace = fwd > adj ? fwd : adj;
  if (f.workspace < 256) f.workspace = 256;
  return f;
}

hipError_t launch_freq_forward(const pa_geometry* g, pa_dtype dt, double f0, double df, int32_t nf, const void* x,
                               void* Y, void* workspace, hipStream_t st) {
  const FreqGeom d = freq_geom(g, f0, df, nf);
  const int64_t m = (int64_t)d.S * nf;
  if (m == 0) return hipSuccess;
  const FreqShape f = freq_shape(d.P, d.S, nf);
  if (d.P == 0) {
    if (dt == PA_F32) freq_zero_kernel<float><<<grid_for(2 * m), kT, 0, st>>>(static_cast<float*>(Y), 2 * m);
    else freq_zero_kernel<double><<<grid_for(2 * m), kT, 0, st>>>(static_cast<double*>(Y), 2 * m);
    return hipGetLastError();
  }
  double2* part = static_cast<double2*>(workspace);
  const int64_t blocks = (int64_t)d.S * f.fwd_fblocks * f.fwd_chunks;
  if (dt == PA_F32) {
    freq_fwd_kernel<float><<<(unsigned)blocks, kT, 0, st>>>(d, static_cast<const float*>(x), part, f.fwd_fblocks,
                                                           f.fwd_chunk_px);
    freq_fwd_reduce_kernel<float><<<grid_for(m), kT, 0, st>>>(d, part, f.fwd_chunks, static_cast<float*>(Y));
  } else {
    freq_fwd_kernel<double><<<(unsigned)blocks, kT, 0, st>>>(d, static_cast<const double*>(x), part, f.fwd_fblocks,
                                                            f.fwd_chunk_px);
    freq_fwd_reduce_kernel<double><<<grid_for(m), kT, 0, st>>>(d, part, f.fwd_chunks, static_cast<double*>(Y));
  }
  return hipGetLastError();
}

hipError_t launch_freq_adjoint(const pa_geometry* g, pa_dtype dt, double f0, double df, int32_t nf, const void* Y,
                               void* x, void* workspace, hipStream_t st) {
  const FreqGeom d = freq_geom(g, f0, df, nf);
  if (d.P == 0) return hipSuccess;
  if ((int64_t)d.S * nf == 0) {
    if (dt == PA_F32) freq_zero_kernel<float><<<grid_for(d.P), kT, 0, st>>>(static_cast<float*>(x), d.P);
    else freq_zero_kernel<double><<<grid_for(d.P), kT, 0, st>>>(static_cast<double*>(x), d.P);
    return hipGetLastError();
  }
  const FreqShape f = freq_shape(d.P, d.S, nf);
  double* part = static_cast<double*>(workspace);
  const int64_t blocks = (int64_t)f.adj_pblocks * f.adj_chunks;
  if (dt == PA_F32) {
    freq_adj_kernel<float><<<(unsigned)blocks, kT, 0, st>>>(d, static_cast<const float*>(Y), part, f.adj_pblocks,
                                                           f.adj_sens);
    freq_adj_reduce_kernel<float><<<grid_for(d.P), kT, 0, st>>>(part, f.adj_chunks, d.P, static_cast<float*>(x));
  } else {
    freq_adj_kernel<double><<<(unsigned)blocks, kT, 0, st>>>(d, static_cast<const double*>(Y), part, f.adj_pblocks,
                                                            f.adj_sens);
    freq_adj_reduce_kernel<double><<<grid_for(d.P), kT, 0, st>>>(part, f.adj_chunks, d.P, static_cast<double*>(x));
  }
  return hipGetLastError();
}

}  // namespace pa
