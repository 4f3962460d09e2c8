// The dense time-domain measurement matrix of Experiment 2 (the paper's kn,
// applied as kn * x and kn' * y in the statement that takes 96.7 % of the
// time in Table 3), materialised on the GPU and applied by HBM-bound
// matrix-vector kernels.  It holds the same operator as pa_forward /
// pa_adjoint, so it serves as a cross-check of the matrix-free path and shows
// the memory wall the matrix-free design removes.
//
// Layout: row m = s * K + k (one measurement), column p (one pixel, ix
// fastest); rows are ld = round_up(P, 32) elements apart and the padding
// columns hold zeros, so every row starts on a 128-byte boundary.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pa_dense.h"

namespace pa {
namespace {

constexpr int kThreads = 256;

// Geometry in SI units as the kernels need it.
struct DenseGeom {
  int32_t ndim, nx, ny, nz, S, K;
  int64_t P, ld;
  double h, cx, cy, cz, dt, t0, c, rmin;
  const double* sensors;   // device [S][ndim], metres
};

template <typename T>
__global__ void __launch_bounds__(kThreads) dense_zero_kernel(T* __restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    a[i] = (T)0;
}

// One thread per (sensor, pixel): its two non-zero entries, (1 - f) / R at
// row k0 and f / R at row k0 + 1 (rows outside the trace are dropped).  No two
// threads write the same entry.  Entries are formed in FP64 and rounded once.
template <typename T>
__global__ void __launch_bounds__(kThreads) dense_taps_kernel(DenseGeom g, T* __restrict__ a) {
  const int64_t n = (int64_t)g.S * g.P;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const int s = (int)(i / g.P);
    const int64_t p = i - (int64_t)s * g.P;
    const int ix = (int)(p % g.nx);
    const int64_t q = p / g.nx;
    const int iy = (int)(q % g.ny);
    const int iz = (int)(q / g.ny);
    const double px = g.cx + ((double)ix - 0.5 * (g.nx - 1)) * g.h;
    const double py = g.cy + ((double)iy - 0.5 * (g.ny - 1)) * g.h;
    const double* sp = g.sensors + (int64_t)s * g.ndim;
    const double dx = px - sp[0], dy = py - sp[1];
    double r2 = dx * dx + dy * dy;
    if (g.ndim == 3) {
      const double pz = g.cz + ((double)iz - 0.5 * (g.nz - 1)) * g.h;
      const double dz = pz - sp[2];
      r2 += dz * dz;
    }
    const double R = fmax(sqrt(r2), g.rmin);
    const double tau = (R / g.c - g.t0) / g.dt;
    const double k0d = floor(tau);
    const double f = tau - k0d;
    const double w = 1.0 / R;
    if (k0d >= 0.0 && k0d <= (double)(g.K - 1)) {
      const int64_t m = (int64_t)s * g.K + (int64_t)k0d;
      a[m * g.ld + p] = (T)(w * (1.0 - f));
    }
    if (k0d + 1.0 >= 0.0 && k0d + 1.0 <= (double)(g.K - 1)) {
      const int64_t m = (int64_t)s * g.K + (int64_t)k0d + 1;
      a[m * g.ld + p] = (T)(w * f);
    }
  }
}

// 16-byte vectors of the matrix element type.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec;
template <> struct Vec<float> { using type = f32x4; static constexpr int n = 4; };
template <> struct Vec<double> { using type = f64x2; static constexpr int n = 2; };

__device__ __forceinline__ double vdot(const f32x4& a, const f32x4& b) {
  return ((double)a.x * (double)b.x + (double)a.y * (double)b.y) + ((double)a.z * (double)b.z + (double)a.w * (double)b.w);
}
__device__ __forceinline__ double vdot(const f64x2& a, const f64x2& b) { return a.x * b.x + a.y * b.y; }

constexpr int kRowsPerWave = 4;
constexpr int kRowsPerBlock = kRowsPerWave * (kThreads / 64);
constexpr int64_t kSplitBelowBlocks = 2048;   // 16-row work-groups below which rows are split over waves
constexpr int kColLoads = 8;                  // A^T: rows in flight per thread

// y = A x: each wave owns four rows and streams them in 16-byte vectors, so
// one load of x feeds four rows.  FP64 accumulation, wave-shuffle reduction
// in a fixed order.  x is read only below P (its padding columns multiply
// zeros, so lanes past P contribute nothing).
template <typename T>
__global__ void __launch_bounds__(kThreads) dense_gemv_kernel(const T* __restrict__ a, const T* __restrict__ x,
                                                              T* __restrict__ y, int64_t M, int64_t P, int64_t ld) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  const int lane = threadIdx.x & 63;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
  double acc[kRowsPerWave] = {0.0, 0.0, 0.0, 0.0};
  const int64_t nv = ld / VN;
  for (int64_t v = lane; v < nv; v += 64) {
    const int64_t p = v * VN;
    V xv;
    if (p + VN <= P) {
      xv = *reinterpret_cast<const V*>(x + p);
    } else {
      T t[VN];
#pragma unroll
      for (int j = 0; j < VN; ++j) t[j] = p + j < P ? x[p + j] : (T)0;
      xv = *reinterpret_cast<const V*>(t);
    }
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      if (row0 + r < M) {
        const V av = __builtin_nontemporal_load(reinterpret_cast<const V*>(a + (row0 + r) * ld) + v);
        acc[r] += vdot(av, xv);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    double s = acc[r];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0 && row0 + r < M) y[row0 + r] = (T)s;
  }
}

// y = A x for matrices with few rows (fewer work-groups of the kernel above
// than the chip has CUs to keep busy): the four waves of a work-group share
// its four rows, wave w taking every fourth 64-vector stretch of columns, so
// four times as many waves stream the matrix.  Each wave's FP64 sums are
// reduced by shuffles, then the four waves' in wave order through LDS.
template <typename T>
__global__ void __launch_bounds__(kThreads) dense_gemv_split_kernel(const T* __restrict__ a, const T* __restrict__ x,
                                                                    T* __restrict__ y, int64_t M, int64_t P,
                                                                    int64_t ld) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  __shared__ double red[4][kRowsPerWave];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsPerWave;
  double acc[kRowsPerWave] = {0.0, 0.0, 0.0, 0.0};
  const int64_t nv = ld / VN;
  for (int64_t v = (int64_t)wave * 64 + lane; v < nv; v += kThreads) {
    const int64_t p = v * VN;
    V xv;
    if (p + VN <= P) {
      xv = *reinterpret_cast<const V*>(x + p);
    } else {
      T t[VN];
#pragma unroll
      for (int j = 0; j < VN; ++j) t[j] = p + j < P ? x[p + j] : (T)0;
      xv = *reinterpret_cast<const V*>(t);
    }
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      if (row0 + r < M) {
        const V av = __builtin_nontemporal_load(reinterpret_cast<const V*>(a + (row0 + r) * ld) + v);
        acc[r] += vdot(av, xv);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    double s = acc[r];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) red[wave][r] = s;
  }
  __syncthreads();
  if (threadIdx.x < kRowsPerWave && row0 + threadIdx.x < M) {
    const int r = threadIdx.x;
    y[row0 + r] = (T)(((red[0][r] + red[1][r]) + red[2][r]) + red[3][r]);
  }
}

// x = A^T y, pass 1: work-group (column block cb, row chunk ch) sums rows
// [ch * rows_per_chunk, ...) of its 256 vectors of columns into FP64 partials
// part[ch][ld].  Each thread owns one 16-byte column vector; y[m] is uniform
// across the work-group.
template <typename T>
__global__ void __launch_bounds__(kThreads) dense_gemvt_partial_kernel(const T* __restrict__ a, const T* __restrict__ y,
                                                                       double* __restrict__ part, int64_t M, int64_t ld,
                                                                       int64_t rows_per_chunk, int col_blocks) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  const int cb = blockIdx.x % col_blocks;
  const int64_t ch = blockIdx.x / col_blocks;
  const int64_t v = (int64_t)cb * kThreads + threadIdx.x;
  const int64_t p = v * VN;
  const int64_t m0 = ch * rows_per_chunk;
  const int64_t m1 = m0 + rows_per_chunk < M ? m0 + rows_per_chunk : M;
  double acc[VN];
#pragma unroll
  for (int j = 0; j < VN; ++j) acc[j] = 0.0;
  if (p < ld) {
    const V* col = reinterpret_cast<const V*>(a) + v;
    const int64_t ldv = ld / VN;
    int64_t m = m0;
    for (; m + kColLoads <= m1; m += kColLoads) {   // kColLoads rows' loads in flight, added in row order
      V av[kColLoads];
#pragma unroll
      for (int u = 0; u < kColLoads; ++u) av[u] = __builtin_nontemporal_load(col + (m + u) * ldv);
#pragma unroll
      for (int u = 0; u < kColLoads; ++u) {
        const double w = (double)y[m + u];
        const T* e = reinterpret_cast<const T*>(&av[u]);
#pragma unroll
        for (int j = 0; j < VN; ++j) acc[j] += (double)e[j] * w;
      }
    }
    for (; m < m1; ++m) {
      const V av = __builtin_nontemporal_load(col + m * ldv);
      const double w = (double)y[m];
      const T* e = reinterpret_cast<const T*>(&av);
#pragma unroll
      for (int j = 0; j < VN; ++j) acc[j] += (double)e[j] * w;
    }
    double* out = part + ch * ld + p;
#pragma unroll
    for (int j = 0; j < VN; ++j) out[j] = acc[j];
  }
}

// x = A^T y, pass 2: x[p] = sum over chunks of part[ch][p], in chunk order.
template <typename T>
__global__ void __launch_bounds__(kThreads) dense_gemvt_reduce_kernel(const double* __restrict__ part, T* __restrict__ x,
                                                                      int64_t P, int64_t ld, int64_t nchunks) {
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < P; p += (int64_t)gridDim.x * kThreads) {
    double s = 0.0;
    for (int64_t ch = 0; ch < nchunks; ++ch) s += part[ch * ld + p];
    x[p] = (T)s;
  }
}

int grid_for(int64_t n) {
  const int64_t g = (n + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

DenseGeom dense_geom(const pa_geometry* g) {
  DenseGeom d;
  d.ndim = g->ndim;
  d.nx = g->nx;
  d.ny = g->ny;
  d.nz = g->ndim == 3 ? g->nz : 1;
  d.S = g->n_sensors;
  d.K = g->n_samples;
  d.P = (int64_t)d.nx * d.ny * d.nz;
  d.ld = dense_ld(d.P);
  d.h = g->h;
  d.cx = g->center[0];
  d.cy = g->center[1];
  d.cz = g->center[2];
  d.dt = g->dt;
  d.t0 = g->t0;
  d.c = g->c;
  d.rmin = g->r_min > 0.0 ? g->r_min : 0.5 * g->h;
  d.sensors = g->sensors;
  return d;
}

}  // namespace

int64_t dense_ld(int64_t P) { return (P + 31) / 32 * 32; }

DenseShape dense_shape(int64_t P, int64_t M) {
  DenseShape s;
  s.ld = dense_ld(P);
  s.col_blocks = (int)((s.ld + 4 * kThreads - 1) / (4 * kThreads));  // covers both vector widths
  // enough work-groups to fill the chip several times over, rows per chunk >= 64
  int64_t want = (4096 + s.col_blocks - 1) / s.col_blocks;
  int64_t maxc = M / 64 > 1 ? M / 64 : 1;
  s.nchunks = want < maxc ? want : maxc;
  if (s.nchunks < 1) s.nchunks = 1;
  s.rows_per_chunk = M > 0 ? (M + s.nchunks - 1) / s.nchunks : 1;
  s.nchunks = M > 0 ? (M + s.rows_per_chunk - 1) / s.rows_per_chunk : 1;
  return s;
}

hipError_t launch_dense_build(const pa_geometry* g, pa_dtype dt, void* a, hipStream_t st) {
  const DenseGeom d = dense_geom(g);
  const int64_t n = (int64_t)d.S * d.K * d.ld;
  const int64_t taps = (int64_t)d.S * d.P;
  if (dt == PA_F32) {
    if (n > 0) dense_zero_kernel<float><<<grid_for(n / 4 + 1), kThreads, 0, st>>>(static_cast<float*>(a), n);
    if (taps > 0) dense_taps_kernel<float><<<grid_for(taps), kThreads, 0, st>>>(d, static_cast<float*>(a));
  } else {
    if (n > 0) dense_zero_kernel<double><<<grid_for(n / 4 + 1), kThreads, 0, st>>>(static_cast<double*>(a), n);
    if (taps > 0) dense_taps_kernel<double><<<grid_for(taps), kThreads, 0, st>>>(d, static_cast<double*>(a));
  }
  return hipGetLastError();
}

hipError_t launch_dense_forward(const pa_geometry* g, pa_dtype dt, const void* a, const void* x, void* y,
                                hipStream_t st) {
  const DenseGeom d = dense_geom(g);
  const int64_t M = (int64_t)d.S * d.K;
  if (M == 0) return hipSuccess;
  const int64_t blocks = (M + kRowsPerBlock - 1) / kRowsPerBlock;
  if (d.P == 0) {   // y = 0
    if (dt == PA_F32) dense_zero_kernel<float><<<grid_for(M), kThreads, 0, st>>>(static_cast<float*>(y), M);
    else dense_zero_kernel<double><<<grid_for(M), kThreads, 0, st>>>(static_cast<double*>(y), M);
    return hipGetLastError();
  }
  if (blocks < kSplitBelowBlocks) {   // too few rows to fill the chip: split each row's columns over four waves
    const int64_t sblocks = (M + kRowsPerWave - 1) / kRowsPerWave;
    if (dt == PA_F32)
      dense_gemv_split_kernel<float><<<(unsigned)sblocks, kThreads, 0, st>>>(
          static_cast<const float*>(a), static_cast<const float*>(x), static_cast<float*>(y), M, d.P, d.ld);
    else
      dense_gemv_split_kernel<double><<<(unsigned)sblocks, kThreads, 0, st>>>(
          static_cast<const double*>(a), static_cast<const double*>(x), static_cast<double*>(y), M, d.P, d.ld);
    return hipGetLastError();
  }
  if (dt == PA_F32)
    dense_gemv_kernel<float><<<(unsigned)blocks, kThreads, 0, st>>>(
        static_cast<const float*>(a), static_cast<const float*>(x), static_cast<float*>(y), M, d.P, d.ld);
  else
    dense_gemv_kernel<double><<<(unsigned)blocks, kThreads, 0, st>>>(
        static_cast<const double*>(a), static_cast<const double*>(x), static_cast<double*>(y), M, d.P, d.ld);
  return hipGetLastError();
}

hipError_t launch_dense_adjoint(const pa_geometry* g, pa_dtype dt, const void* a, const void* y, void* x,
                                void* workspace, hipStream_t st) {
  const DenseGeom d = dense_geom(g);
  const int64_t M = (int64_t)d.S * d.K;
  if (d.P == 0) return hipSuccess;
  if (M == 0) {   // x = 0
    if (dt == PA_F32) dense_zero_kernel<float><<<grid_for(d.P), kThreads, 0, st>>>(static_cast<float*>(x), d.P);
    else dense_zero_kernel<double><<<grid_for(d.P), kThreads, 0, st>>>(static_cast<double*>(x), d.P);
    return hipGetLastError();
  }
  const DenseShape s = dense_shape(d.P, M);
  double* part = static_cast<double*>(workspace);
  const int64_t vn = dt == PA_F32 ? 4 : 2;
  const int cbs = (int)((d.ld / vn + kThreads - 1) / kThreads);
  const int64_t blocks = (int64_t)cbs * s.nchunks;
  if (dt == PA_F32) {
    dense_gemvt_partial_kernel<float><<<(unsigned)blocks, kThreads, 0, st>>>(
        static_cast<const float*>(a), static_cast<const float*>(y), part, M, d.ld, s.rows_per_chunk, cbs);
    dense_gemvt_reduce_kernel<float><<<grid_for(d.P), kThreads, 0, st>>>(part, static_cast<float*>(x), d.P, d.ld,
                                                                         s.nchunks);
  } else {
    dense_gemvt_partial_kernel<double><<<(unsigned)blocks, kThreads, 0, st>>>(
        static_cast<const double*>(a), static_cast<const double*>(y), part, M, d.ld, s.rows_per_chunk, cbs);
    dense_gemvt_reduce_kernel<double><<<grid_for(d.P), kThreads, 0, st>>>(part, static_cast<double*>(x), d.P, d.ld,
                                                                          s.nchunks);
  }
  return hipGetLastError();
}

}  // namespace pa
