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

#include "pa_device.h"
#include "pa_kernels.h"

namespace pa {

namespace {

using dev::block_sum;


constexpr float kInactiveCmin = 1.0f;

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Work-groups are dealt round-robin to the 8 XCDs (block b -> XCD b % 8).
  // Give each XCD a contiguous run of tiles so neighbouring tiles, which read
  // overlapping trace windows, share one L2.
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + idx;
}

__device__ __forceinline__ size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

// ---------------------------------------------------------------------------
// Per (tile, sensor) constants.
//
// FP32 path ("tile-local delay").  tau ~ 2000 samples has an FP32 spacing of
// 1.2e-4, too coarse for the interpolation fraction.  Instead each (tile,
// sensor) pair gets, in FP64, the sensor-to-tile-centre vector D (sample
// units) and an integer reference kr = round(|D|).  For a pixel at offset o
// from the tile centre,
//   num = R^2 - kr^2 = (|D|^2 - kr^2) + 2 D.o + |o|^2
// is formed in FP32 from small terms, and R - kr follows from one Newton step
// on d (d + 2 kr) = num starting at the FP32 estimate R^2 * rsq(R^2) - kr.
// The result is accurate to ~1e-6 samples.
struct SC32 {
  float E;      // |D|^2 - kr^2
  float DX2, DY2, DZ2;  // 2 D
  float KRN;    // -kr
  float KR2N;   // -2 kr
  float KR2;    // kr^2
  float CMIN;   // rmin^2 - kr^2 (distance clamp, in num units)
  int BASE;     // byte offset of sample (kr - t0i) in this sensor's LDS row
  int act;      // 0: sensor contributes nothing to this tile
  float HALF;   // 0.5 (active) or 0 (inactive): weight multiplier
  int pad;
};
static_assert(sizeof(SC32) == 48, "SC32 layout");

// FP64 path: plain distance arithmetic in double.
struct SC64 {
  double DX, DY, DZ;  // D
  double KR;          // kr
  double RMIN2;       // rmin^2
  double ACT;         // 1 or 0: weight multiplier
  double T0F;         // t0 / dt - floor(t0 / dt)
  int BASE;           // byte offset of sample (kr - t0i) in this sensor's LDS row
  int act;
};
static_assert(sizeof(SC64) == 64, "SC64 layout");

template <typename T> struct SCOf;
template <> struct SCOf<float> { using type = SC32; };
template <> struct SCOf<double> { using type = SC64; };

// Offsets of one pixel of a base tile from the tile centre, sample units.
struct Pix32 { float ox, oy, oz, q; };
struct Pix64 { double ox, oy, oz, pad; };
template <typename T> struct PixOf;
template <> struct PixOf<float> { using type = Pix32; };
template <> struct PixOf<double> { using type = Pix64; };

template <int ND>
__device__ __forceinline__ void pix_offsets(const OpParams& P, int lx, int ly, int lz, double o[3]) {
  o[0] = ((double)lx - 0.5 * (Tile<ND>::X - 1)) * P.hs;
  o[1] = ((double)ly - 0.5 * (Tile<ND>::Y - 1)) * P.hs;
  o[2] = ND == 3 ? ((double)lz - 0.5 * (Tile<ND>::Z - 1)) * P.hs : 0.0;
}

template <int ND>
__device__ __forceinline__ void make_pix(const OpParams& P, int lx, int ly, int lz, Pix32& p) {
  double o[3];
  pix_offsets<ND>(P, lx, ly, lz, o);
  p.ox = (float)o[0];
  p.oy = (float)o[1];
  p.oz = (float)o[2];
  p.q = (float)(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
}

template <int ND>
__device__ __forceinline__ void make_pix(const OpParams& P, int lx, int ly, int lz, Pix64& p) {
  double o[3];
  pix_offsets<ND>(P, lx, ly, lz, o);
  p.ox = o[0];
  p.oy = o[1];
  p.oz = o[2];
  p.pad = 0.0;
}

// Centre of base tile (bx, by, bz), sample units.
template <int ND>
__device__ __forceinline__ void tile_ref(const OpParams& P, int bx, int by, int bz, double r[3]) {
  r[0] = P.org[0] + ((double)bx * Tile<ND>::X + 0.5 * (Tile<ND>::X - 1)) * P.hs;
  r[1] = P.org[1] + ((double)by * Tile<ND>::Y + 0.5 * (Tile<ND>::Y - 1)) * P.hs;
  r[2] = ND == 3 ? P.org[2] + ((double)bz * Tile<ND>::Z + 0.5 * (Tile<ND>::Z - 1)) * P.hs : 0.0;
}

template <int ND>
__device__ __forceinline__ void sensor_pos(const OpParams& P, int s, double sp[3]) {
  sp[0] = P.sensors[(size_t)s * ND + 0] * P.inv_cdt;
  sp[1] = P.sensors[(size_t)s * ND + 1] * P.inv_cdt;
  sp[2] = ND == 3 ? P.sensors[(size_t)s * ND + 2] * P.inv_cdt : 0.0;
}

// First sample of the LDS window that covers every tap of every pixel centre
// in the box [lo, hi] (sample units) for a sensor at sp.
template <int ND>
__device__ __forceinline__ int window_lo(const OpParams& P, const double lo[3], const double hi[3],
                                         const double sp[3], bool* in_trace, int width) {
  double dmin2 = 0.0, dmax2 = 0.0;
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    double e = fmax(fmax(lo[a] - sp[a], sp[a] - hi[a]), 0.0);
    dmin2 += e * e;
    double f = fmax(fabs(lo[a] - sp[a]), fabs(hi[a] - sp[a]));
    dmax2 += f * f;
  }
  double dmin = fmax(sqrt(dmin2), P.rmin);
  double dmax = fmax(sqrt(dmax2), P.rmin);
  double tmin = dmin - (double)P.t0i - P.t0fd;
  double tmax = dmax - (double)P.t0i - P.t0fd;
  *in_trace = tmax >= -2.0 && tmin <= (double)P.K + 1.0 && dmax < 4.0e6;
  double klo = floor(tmin) - 1.0;
  klo = fmin(fmax(klo, -4.0 * width), (double)P.K + 4.0);  // keep integer conversions in range
  return (int)klo;
}

template <int ND>
__device__ __forceinline__ void make_sc(const OpParams& P, const double ref[3], const double sp[3], int klo,
                                        int row_elems, bool active, SC32& c) {
  double dx = ref[0] - sp[0], dy = ref[1] - sp[1], dz = ND == 3 ? ref[2] - sp[2] : 0.0;
  double ra2 = dx * dx + dy * dy + dz * dz;
  double kr = rint(sqrt(ra2));
  if (!active) {  // benign constants: bounded delay, zero weight
    c.E = 0.f; c.DX2 = 0.f; c.DY2 = 0.f; c.DZ2 = 0.f; c.KRN = 0.f; c.KR2N = 0.f; c.KR2 = 0.f;
    c.CMIN = kInactiveCmin; c.BASE = row_elems * 4; c.act = 0; c.HALF = 0.f;
    return;
  }
  c.E = (float)(ra2 - kr * kr);
  c.DX2 = (float)(2.0 * dx);
  c.DY2 = (float)(2.0 * dy);
  c.DZ2 = (float)(2.0 * dz);
  c.KRN = (float)(-kr);
  c.KR2N = (float)(-2.0 * kr);
  c.KR2 = (float)(kr * kr);
  c.CMIN = (float)(P.rmin * P.rmin - kr * kr);
  c.BASE = ((int)kr - P.t0i - klo + row_elems) * 4;
  c.act = 1;
  c.HALF = 0.5f;
}

template <int ND>
__device__ __forceinline__ void make_sc(const OpParams& P, const double ref[3], const double sp[3], int klo,
                                        int row_elems, bool active, SC64& c) {
  double dx = ref[0] - sp[0], dy = ref[1] - sp[1], dz = ND == 3 ? ref[2] - sp[2] : 0.0;
  double kr = active ? rint(sqrt(dx * dx + dy * dy + dz * dz)) : 0.0;
  c.DX = active ? dx : 0.0;
  c.DY = active ? dy : 0.0;
  c.DZ = active ? dz : 0.0;
  c.KR = kr;
  c.RMIN2 = active ? P.rmin * P.rmin : 1.0;
  c.ACT = active ? 1.0 : 0.0;
  c.T0F = P.t0fd;
  c.BASE = ((int)kr - P.t0i - klo + row_elems) * 8;
  c.act = active ? 1 : 0;
}

// The per-pair arithmetic.  Returns the byte offset of tap k0 in LDS, the
// fraction f and the tap weight in kernel units (FP32: 1 / (2R); FP64: 1 / R).
template <int ND, bool FRAC>
__device__ __forceinline__ void phase(const SC32& c, const Pix32& px, float t0f, int& kbyte, float& f, float& wt) {
  float t = px.q + c.E;
  float num = fmaf(px.oy, c.DY2, t);
  if (ND == 3) num = fmaf(px.oz, c.DZ2, num);
  num = fmaf(px.ox, c.DX2, num);
  num = fmaxf(num, c.CMIN);
  const float R2 = num + c.KR2;
  const float w = __builtin_amdgcn_rsqf(R2);
  const float da = fmaf(R2, w, c.KRN);       // R - kr, FP32 estimate
  const float r1 = fmaf(c.KR2N, da, num);
  const float r = fmaf(-da, da, r1);         // num - da (da + 2 kr)
  wt = c.HALF * w;                           // 1 / (2R)
  float d = fmaf(r, wt, da);                 // Newton-corrected R - kr
  if (FRAC) d = d - t0f;
  f = __builtin_amdgcn_fractf(d);           // d - floor(d), exact
  kbyte = (int)floorf(d) * 4 + c.BASE;
}

template <int ND, bool FRAC>
__device__ __forceinline__ void phase(const SC64& c, const Pix64& px, float, int& kbyte, double& f, double& wt) {
  const double dx = px.ox + c.DX;
  const double dy = px.oy + c.DY;
  double R2 = dx * dx + dy * dy;
  if (ND == 3) {
    const double dz = px.oz + c.DZ;
    R2 = R2 + dz * dz;
  }
  R2 = fmax(R2, c.RMIN2);
  const double R = sqrt(R2);
  wt = c.ACT / R;
  double d = R - c.KR;
  if (FRAC) d = d - c.T0F;
  const double fl = floor(d);
  f = d - fl;
  kbyte = (int)fl * 8 + c.BASE;
}

// Atomic add through an LDS byte address held in an integer register.
template <typename T>
__device__ __forceinline__ void lds_add(T* addr, T v) {
  __hip_atomic_fetch_add(reinterpret_cast<__attribute__((address_space(3))) T*>(static_cast<unsigned>(reinterpret_cast<size_t>(addr))),
                         v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Load through an LDS byte address held in an integer register.
template <typename T>
__device__ __forceinline__ T lds_load(const T* addr) {
  return *reinterpret_cast<const __attribute__((address_space(3))) T*>(
      static_cast<unsigned>(reinterpret_cast<size_t>(addr)));
}

}  // namespace

// ---------------------------------------------------------------------------
// A^T: one work-group per base tile, one pixel per lane.  Sensors are taken in
// chunks: the chunk's per-sensor constants and each sensor's trace window
// (the samples any pixel of the tile can reach, zero outside 0..K-1) are
// staged in LDS, then every lane gathers its two taps per sensor from LDS.
// With CG the epilogue also performs x += alpha p, s = A^T r - lambda x and the
// FP64 partial sums of ||s||^2 and ||x||^2.
template <typename T, int ND, bool FRAC, bool CG>
__global__ void __launch_bounds__(kBlock) bp_kernel(OpParams P, const T* __restrict__ y, T* __restrict__ out,
                                                     T* __restrict__ xcg, const T* __restrict__ pcg,
                                                     const double* __restrict__ alpha, double lambda,
                                                     double* __restrict__ part_s, double* __restrict__ part_x) {
  using SC = typename SCOf<T>::type;
  using PX = typename PixOf<T>::type;
  constexpr int TX = Tile<ND>::X, TY = Tile<ND>::Y, TZ = Tile<ND>::Z;
  extern __shared__ __align__(16) unsigned char smem[];
  SC* sct = reinterpret_cast<SC*>(smem);
  int* klo_s = reinterpret_cast<int*>(smem + align16((size_t)P.sc * sizeof(SC)));
  T* win = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(klo_s) + align16((size_t)P.sc * 4));
  __shared__ double red[4];

  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = tile % P.ntile[0];
  const int by = (tile / P.ntile[0]) % P.ntile[1];
  const int bz = tile / (P.ntile[0] * P.ntile[1]);
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
  const int ix = bx * TX + lx, iy = by * TY + ly, iz = bz * TZ + lz;
  const bool valid = ix < P.nx && iy < P.ny && iz < P.nz;

  double ref[3], lo[3], hi[3];
  tile_ref<ND>(P, bx, by, bz, ref);
  {
    const int T3[3] = {TX, TY, TZ};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double half = 0.5 * (T3[a] - 1) * P.hs;
      lo[a] = ref[a] - half;
      hi[a] = ref[a] + half;
    }
  }
  PX px;
  make_pix<ND>(P, lx, ly, lz, px);
  const float t0f = P.t0f;

  T acc = 0;
  for (int s0 = 0; s0 < P.S; s0 += P.sc) {
    const int nsc = min(P.sc, P.S - s0);
    if (tid < nsc) {
      double sp[3];
      sensor_pos<ND>(P, s0 + tid, sp);
      bool in_trace;
      const int kl = window_lo<ND>(P, lo, hi, sp, &in_trace, P.wp);
      SC c;
      make_sc<ND>(P, ref, sp, kl, tid * P.wp, in_trace, c);
      c.BASE += (int)(size_t)win;  // absolute LDS byte address of the row's reference sample
      sct[tid] = c;
      klo_s[tid] = in_trace ? kl : P.K + 8;  // inactive rows stage zeros
    }
    __syncthreads();
    const int tot = nsc * P.wp;
    for (int e = tid; e < tot; e += kBlock) {
      const int j = (int)__umulhi((unsigned)e, P.wp_magic);
      const int k = klo_s[j] + (e - j * P.wp);
      T v = 0;
      if (k >= 0 && k < P.K) v = y[(size_t)(s0 + j) * P.K + k];
      win[e] = v;
    }
    __syncthreads();
    // Sensors whose arrivals miss the trace carry zero weight and a bounded
    // delay into a zero row, so the loop needs no per-sensor test.
    // Four sensors per step: four delays, then four independent window
    // reads, then the sums in sensor order (the order never changes).
    int j = 0;
    for (; j + 4 <= nsc; j += 4) {
      int kb[4];
      T f[4], wt[4], y0[4], y1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) phase<ND, FRAC>(sct[j + u], px, t0f, kb[u], f[u], wt[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T* tap = reinterpret_cast<const T*>(static_cast<size_t>(kb[u]));
        y0[u] = lds_load(tap);
        y1[u] = lds_load(tap + 1);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma(wt[u], fma(f[u], y1[u] - y0[u], y0[u]), acc);
    }
    for (; j < nsc; ++j) {
      int kb;
      T f, wt;
      phase<ND, FRAC>(sct[j], px, t0f, kb, f, wt);
      const T* tap = reinterpret_cast<const T*>(static_cast<size_t>(kb));
      const T y0 = lds_load(tap);
      const T y1 = lds_load(tap + 1);
      acc = fma(wt, fma(f, y1 - y0, y0), acc);
    }
    __syncthreads();
  }

  const size_t idx = ((size_t)iz * P.ny + iy) * P.nx + ix;
  const T scale = sizeof(T) == 4 ? (T)P.out_scale : (T)P.out_scale_d;
  if (!CG) {
    if (valid) out[idx] = acc * scale;
    return;
  }
  double ss = 0.0, xx = 0.0;
  if (valid) {
    const double a = *alpha;
    double xo = (double)xcg[idx];
    if (a != 0.0) xo += a * (double)pcg[idx];
    const T xn = (T)xo;
    const T sn = (T)((double)(acc * scale) - lambda * (double)xn);
    out[idx] = sn;
    xcg[idx] = xn;
    ss = (double)sn * (double)sn;
    xx = (double)xn * (double)xn;
  }
  ss = block_sum(ss, red);
  xx = block_sum(xx, red);
  if (tid == 0) {
    part_s[blockIdx.x] = ss;
    part_x[blockIdx.x] = xx;
  }
}

// ---------------------------------------------------------------------------
// A: one work-group per (forward tile, chunk of 64 sensors); lane = sensor,
// wave w walks base tiles w, w+4, ... of the forward tile one pixel at a time
// (the pixel is uniform across the wave).  Each lane scatters its two taps
// into its own sensor's LDS histogram row, so the lanes of one ds_add never
// collide on an address.  The rows are then added into y with global atomics
// (y must be zero on entry).
template <typename T, int ND, bool FRAC>
__global__ void __launch_bounds__(kBlock) fp_kernel(OpParams P, const T* __restrict__ x, T* __restrict__ y) {
  using SC = typename SCOf<T>::type;
  using PX = typename PixOf<T>::type;
  constexpr int TX = Tile<ND>::X, TY = Tile<ND>::Y, TZ = Tile<ND>::Z;
  constexpr int NS = kSensorsPerFwdBlock;
  extern __shared__ __align__(16) unsigned char smem[];
  T* hist = reinterpret_cast<T*>(smem);
  unsigned char* p1 = smem + align16((size_t)NS * P.wpa * sizeof(T));
  PX* pixtab = reinterpret_cast<PX*>(p1);
  T* xs = reinterpret_cast<T*>(p1 + (size_t)kBlock * sizeof(PX));
  int* klo_a = reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(xs) + align16((size_t)P.nsub * kBlock * sizeof(T)));

  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = b % P.n_chunks;
  const int at = b / P.n_chunks;
  const int ax = at % P.natile[0];
  const int ay = (at / P.natile[0]) % P.natile[1];
  const int az = at / (P.natile[0] * P.natile[1]);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
  const int s = chunk * NS + lane;
  const bool s_ok = s < P.S;

  // pixel offsets of a base tile (same for every base tile) and the forward tile's x values
  {
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    make_pix<ND>(P, lx, ly, lz, pixtab[tid]);
    for (int m = 0; m < P.nsub; ++m) {
      const int bx = ax * P.msub[0] + m % P.msub[0];
      const int by = ay * P.msub[1] + (m / P.msub[0]) % P.msub[1];
      const int bz = az * P.msub[2] + m / (P.msub[0] * P.msub[1]);
      const int ix = bx * TX + lx, iy = by * TY + ly, iz = bz * TZ + lz;
      T v = 0;
      if (ix < P.nx && iy < P.ny && iz < P.nz) v = x[((size_t)iz * P.ny + iy) * P.nx + ix];
      xs[m * kBlock + tid] = v;
    }
  }
  // this lane's sensor and its window over the whole forward tile
  double sp[3];
  sensor_pos<ND>(P, s_ok ? s : P.S - 1, sp);
  bool in_trace;
  int kl;
  {
    double lo[3], hi[3];
    const int T3[3] = {TX, TY, TZ};
    double r0[3];
    tile_ref<ND>(P, ax * P.msub[0], ay * P.msub[1], az * P.msub[2], r0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = r0[a] - 0.5 * (T3[a] - 1) * P.hs;
      hi[a] = lo[a] + (P.msub[a] * T3[a] - 1) * P.hs;
    }
    if (ND == 2) { lo[2] = 0.0; hi[2] = 0.0; }
    kl = window_lo<ND>(P, lo, hi, sp, &in_trace, P.wpa);
  }
  const bool active = s_ok && in_trace;
  if (wave == 0) klo_a[lane] = active ? kl : P.K + 8;
  for (int e = tid; e < NS * P.wpa; e += kBlock) hist[e] = 0;
  __syncthreads();

  const float t0f = P.t0f;
  for (int m = wave; m < P.nsub; m += 4) {
    const int bx = ax * P.msub[0] + m % P.msub[0];
    const int by = ay * P.msub[1] + (m / P.msub[0]) % P.msub[1];
    const int bz = az * P.msub[2] + m / (P.msub[0] * P.msub[1]);
    const int nlx = __builtin_amdgcn_readfirstlane(min(TX, P.nx - bx * TX));
    const int nly = __builtin_amdgcn_readfirstlane(min(TY, P.ny - by * TY));
    const int nlz = __builtin_amdgcn_readfirstlane(min(TZ, P.nz - bz * TZ));
    if (nlx <= 0 || nly <= 0 || nlz <= 0) continue;
    double ref[3];
    tile_ref<ND>(P, bx, by, bz, ref);
    SC c;
    make_sc<ND>(P, ref, sp, kl, lane * P.wpa, active, c);
    c.BASE += (int)(size_t)hist;  // absolute LDS byte address
    asm volatile("" : "+v"(c.BASE));  // keep "k * 4 + BASE" a single shift-add
    const T* xm = xs + m * kBlock;
    for (int lz = 0; lz < nlz; ++lz) {
      for (int ly = 0; ly < nly; ++ly) {
        const int rowp = (lz * TY + ly) * TX;
#pragma unroll 2
        for (int lx = 0; lx < nlx; ++lx) {
          const PX px = pixtab[rowp + lx];
          const T xp = xm[rowp + lx];
          int kb;
          T f, wt;
          phase<ND, FRAC>(c, px, t0f, kb, f, wt);
          const T v = wt * xp;
          const T a1 = v * f;
          const T a0 = v - a1;
          T* bin = reinterpret_cast<T*>(static_cast<size_t>(kb));
          lds_add(bin, a0);
          lds_add(bin + 1, a1);
        }
      }
    }
  }
  __syncthreads();

  const T scale = sizeof(T) == 4 ? (T)P.out_scale : (T)P.out_scale_d;
  for (int j = wave; j < NS; j += 4) {
    const int sj = chunk * NS + j;
    if (sj >= P.S) break;
    const int k0 = klo_a[j];
    T* row = y + (size_t)sj * P.K;
    for (int i = lane; i < P.wpa; i += 64) {
      const int k = k0 + i;
      const T v = hist[j * P.wpa + i];
      if (v != (T)0 && k >= 0 && k < P.K) unsafeAtomicAdd(row + k, v * scale);
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.

namespace {

template <typename T, int ND, bool FRAC, bool CG>
hipError_t launch_bp_t(const Plan& pl, const T* y, T* out, const CgArgs* cg, hipStream_t st) {
  const OpParams& P = pl.op;
  if (CG)
    bp_kernel<T, ND, FRAC, CG><<<pl.bp_grid, kBlock, pl.bp_lds, st>>>(
        P, y, out, static_cast<T*>(cg->x), static_cast<const T*>(cg->p), cg->alpha, cg->lambda, cg->part_s, cg->part_x);
  else
    bp_kernel<T, ND, FRAC, CG><<<pl.bp_grid, kBlock, pl.bp_lds, st>>>(P, y, out, nullptr, nullptr, nullptr, 0.0,
                                                                      nullptr, nullptr);
  return hipGetLastError();
}

template <typename T, int ND, bool CG>
hipError_t launch_bp_f(const Plan& pl, const T* y, T* out, const CgArgs* cg, hipStream_t st) {
  return pl.op.t0f != 0.0f ? launch_bp_t<T, ND, true, CG>(pl, y, out, cg, st)
                           : launch_bp_t<T, ND, false, CG>(pl, y, out, cg, st);
}

template <typename T, int ND, bool FRAC>
hipError_t launch_fp_t(const Plan& pl, const T* x, T* y, hipStream_t st) {
  fp_kernel<T, ND, FRAC><<<pl.fp_grid, kBlock, pl.fp_lds, st>>>(pl.op, x, y);
  return hipGetLastError();
}

template <typename T, int ND>
hipError_t launch_fp_f(const Plan& pl, const T* x, T* y, hipStream_t st) {
  return pl.op.t0f != 0.0f ? launch_fp_t<T, ND, true>(pl, x, y, st) : launch_fp_t<T, ND, false>(pl, x, y, st);
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

hipError_t launch_forward_accumulate(const Plan& pl, const void* x, void* y, hipStream_t st) {
  if (pl.fp_grid == 0) return hipSuccess;
  if (pl.dtype == PA_F32) {
    auto xx = static_cast<const float*>(x);
    auto yy = static_cast<float*>(y);
    return pl.ndim == 2 ? launch_fp_f<float, 2>(pl, xx, yy, st) : launch_fp_f<float, 3>(pl, xx, yy, st);
  }
  auto xx = static_cast<const double*>(x);
  auto yy = static_cast<double*>(y);
  return pl.ndim == 2 ? launch_fp_f<double, 2>(pl, xx, yy, st) : launch_fp_f<double, 3>(pl, xx, yy, st);
}

}  // namespace pa
