// Device code of the operator kernels: per-pair delay arithmetic, LDS
// layouts and the kernel bodies, shared by the single-frame kernels
// (pa_ops.hip) and the batched kernels (pa_batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "pa_device.h"
#include "pa_kernels.h"
#include "pa_plan.h"

namespace pa {

namespace {

using dev::block_sum;



__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Work-groups are dealt round-robin to the 8 XCDs (block b -> XCD b % 8).
  // Give each XCD a contiguous run of tiles so neighbouring tiles, which read
  // overlapping trace windows, share one L2.
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + idx;
}

// ---------------------------------------------------------------------------
// Per (tile, sensor) constants.
//
// FP32 path ("tile-local delay").  tau ~ 2000 samples has an FP32 spacing of
// 1.2e-4, too coarse for the interpolation fraction.  Instead each (tile,
// sensor) pair gets, in FP64, the sensor-to-tile-centre vector D (sample
// units) and an integer reference kr = round(|D|).  For a pixel at offset o
// from the tile centre,
//   num = R^2 - kr^2 = (|D|^2 - kr^2) + 2 D.o + |o|^2
// is formed in FP32 from small terms (as num / 2, every term halved, which
// is exact), and R - kr follows from one Newton step on d (d + 2 kr) = num
// starting at the FP32 estimate R^2 * rsq(R^2) - kr.  The result is accurate
// to ~1e-6 samples.  The pixel enters through its offset u in pixel pitches
// (o = hs u; half-integers, exact in FP32), so its constants are the same
// for every plan: D.o = u.(hs D) and |o|^2 / 2 = (hs^2 / 2) |u|^2.
struct SC32 {
  float E;      // (|D|^2 - kr^2) / 2
  float DXH, DYH, DZH;  // hs D
  float KRN;    // -kr
  float KR2;    // kr^2
  float CMIN;   // (rmin^2 - kr^2) / 2: the distance clamp in num / 2 units (never reached by far pairs)
  int BASE;     // byte offset of sample (kr - t0i) in this sensor's LDS row
  int act;      // 0: sensor contributes nothing to this tile
  int pad[3];
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

// Offset of one pixel of a base tile from the tile centre: FP32, in pixel
// pitches (ux, uy, uz) with uq = |u|^2; FP64, in sample units.
struct Pix32 { float ux, uy, uz, uq; };
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
__host__ __device__ constexpr Pix32 unit_pix(int lx, int ly, int lz) {
  const float ux = (float)lx - 0.5f * (Tile<ND>::X - 1);
  const float uy = (float)ly - 0.5f * (Tile<ND>::Y - 1);
  const float uz = ND == 3 ? (float)lz - 0.5f * (Tile<ND>::Z - 1) : 0.f;
  return Pix32{ux, uy, uz, ux * ux + uy * uy + uz * uz};   // all exact
}

template <int ND>
__device__ __forceinline__ void make_pix(const OpParams&, int lx, int ly, int lz, Pix32& p) {
  p = unit_pix<ND>(lx, ly, lz);
}

// The unit offsets of a base tile's pixels in pixel order (lx fastest), in
// constant memory: a wave-uniform index reads them with scalar loads.  Four
// entries of slack past the tile: a loop may read four pixels ahead.
struct PixTable {
  Pix32 p[kBlock + 4];
};
template <int ND>
constexpr PixTable make_pix_table() {
  PixTable t{};
  for (int i = 0; i < kBlock; ++i)
    t.p[i] = unit_pix<ND>(i % Tile<ND>::X, (i / Tile<ND>::X) % Tile<ND>::Y, i / (Tile<ND>::X * Tile<ND>::Y));
  return t;
}
__constant__ constexpr PixTable kPixTable2 = make_pix_table<2>();
__constant__ constexpr PixTable kPixTable3 = make_pix_table<3>();
template <int ND>
__device__ __forceinline__ const Pix32* pix_table() {
  return ND == 2 ? kPixTable2.p : kPixTable3.p;
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
                                         const double sp[3], bool* in_trace, int width, double* dmin_out = nullptr) {
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
  if (dmin_out) *dmin_out = dmin;
  double tmin = dmin - (double)P.t0i - P.t0fd;
  double tmax = dmax - (double)P.t0i - P.t0fd;
  *in_trace = tmax >= -2.0 && tmin <= (double)P.K + 1.0 && dmax < 4.0e6;
  double klo = floor(tmin) - 1.0;
  klo = fmin(fmax(klo, -4.0 * width), (double)P.K + 4.0);  // keep integer conversions in range
  return (int)klo;
}

template <int ND>
__device__ __forceinline__ void make_sc(const OpParams& P, const double ref[3], const double sp[3], int klo,
                                        int row_elems, int esz, bool active, SC32& c) {
  double dx = ref[0] - sp[0], dy = ref[1] - sp[1], dz = ND == 3 ? ref[2] - sp[2] : 0.0;
  double ra2 = dx * dx + dy * dy + dz * dz;
  double kr = rint(sqrt(ra2));
  // Benign constants: num = |o|^2 + 1 >= 1, a delay of at most |o| + 1 and a
  // finite weight; the caller zeroes the contribution (the adjoint stages a
  // zero row for the sensor, the partial-row forward gives the pair a zero
  // fixed-point scale).
  if (!active) {
    c.E = 0.5f; c.DXH = 0.f; c.DYH = 0.f; c.DZH = 0.f; c.KRN = 0.f; c.KR2 = 0.f;
    c.CMIN = 0.5f; c.BASE = row_elems * esz; c.act = 0;
    return;
  }
  c.E = (float)(0.5 * (ra2 - kr * kr));
  c.DXH = (float)(P.hs * dx);
  c.DYH = (float)(P.hs * dy);
  c.DZH = (float)(P.hs * dz);
  c.KRN = (float)(-kr);
  c.KR2 = (float)(kr * kr);
  c.CMIN = (float)(0.5 * (P.rmin * P.rmin - kr * kr));
  c.BASE = ((int)kr - P.t0i - klo + row_elems) * esz;
  c.act = 1;
}

template <int ND>
__device__ __forceinline__ void make_sc(const OpParams& P, const double ref[3], const double sp[3], int klo,
                                        int row_elems, int esz, bool active, SC64& c) {
  double dx = ref[0] - sp[0], dy = ref[1] - sp[1], dz = ND == 3 ? ref[2] - sp[2] : 0.0;
  double kr = active ? rint(sqrt(dx * dx + dy * dy + dz * dz)) : 0.0;
  c.DX = active ? dx : 0.0;
  c.DY = active ? dy : 0.0;
  c.DZ = active ? dz : 0.0;
  c.KR = kr;
  c.RMIN2 = active ? P.rmin * P.rmin : 1.0;
  c.ACT = active ? 1.0 : 0.0;
  c.T0F = P.t0fd;
  c.BASE = ((int)kr - P.t0i - klo + row_elems) * esz;
  c.act = active ? 1 : 0;
}

// FP64 sensor vector and reference of a "near" (tile, sensor) pair, used by
// the FP32 kernels: when a sensor lies within a few tile half-diagonals of
// the tile, R can be small against the tile-local terms of num, so the delay
// and weight of such pairs are formed from FP64 coordinates instead.
struct Near32 {
  double DX, DY, DZ, KR;
};
static_assert(sizeof(Near32) == 32, "Near32 layout");

// The per-pair arithmetic.  Returns the LDS byte address of tap k0 (rows of
// ESZ-byte entries), the fraction f and the tap weight 1 / R.  Far pairs
// never reach the distance clamp (the near radius covers r_min), and
// inactive ones have num >= 1, so the FP32 kernels leave the max instruction
// out (CLAMP = false): either choice gives the same taps.  hs2h = hs^2 / 2.
template <int ND, bool FRAC, int ESZ, bool CLAMP, typename C>
__device__ __forceinline__ void phase32(const C& c, float cmin, const Pix32& px, float t0f, float hs2h,
                                        int& kbyte, float& f, float& w) {
  float t = fmaf(px.uq, hs2h, c.E);
  float nh = fmaf(px.uy, c.DYH, t);          // num / 2
  if (ND == 3) nh = fmaf(px.uz, c.DZH, nh);
  nh = fmaf(px.ux, c.DXH, nh);
  if (CLAMP) nh = fmaxf(nh, cmin);
  const float R2 = fmaf(2.0f, nh, c.KR2);    // num + kr^2 (the doubling is exact)
  w = __builtin_amdgcn_rsqf(R2);             // 1 / R
  const float da = fmaf(R2, w, c.KRN);       // R - kr, FP32 estimate
  const float h = fmaf(-0.5f, da, c.KRN);    // -(kr + da / 2)
  const float rh = fmaf(da, h, nh);          // (num - da (da + 2 kr)) / 2 = (R^2 - (kr + da)^2) / 2
  float d = fmaf(rh, w, da);                 // Newton-corrected R - kr
  if (FRAC) d = d - t0f;
  f = __builtin_amdgcn_fractf(d);           // d - floor(d), exact
  kbyte = (int)floorf(d) * ESZ + c.BASE;
}

template <int ND, bool FRAC, int ESZ, bool CLAMP = true>
__device__ __forceinline__ void phase(const SC32& c, const Pix32& px, float t0f, float hs2h, int& kbyte, float& f,
                                      float& w) {
  phase32<ND, FRAC, ESZ, CLAMP>(c, c.CMIN, px, t0f, hs2h, kbyte, f, w);
}

// Forward operator: far pairs only (active, no clamp reached).
template <int ND, bool FRAC, int ESZ, bool CLAMP = false>
__device__ __forceinline__ void phase(const FpSC32& c, const Pix32& px, float t0f, float hs2h, int& kbyte, float& f,
                                      float& w) {
  phase32<ND, FRAC, ESZ, false>(c, 0.f, px, t0f, hs2h, kbyte, f, w);
}

__device__ __forceinline__ FpSC32 fp_sc(const SC32& c) {
  FpSC32 o;
  o.E = c.E;
  o.DXH = c.DXH;
  o.DYH = c.DYH;
  o.DZH = c.DZH;
  o.KRN = c.KRN;
  o.KR2 = c.KR2;
  o.BASE = c.BASE;
  return o;
}
__device__ __forceinline__ SC64 fp_sc(const SC64& c) { return c; }

// FP32 kernels, near pairs: delay and weight from FP64 coordinates.
template <int ND, bool FRAC, int ESZ>
__device__ __forceinline__ void phase_near(const Near32& n, const double o[3], double rmin2, double t0fd, int base,
                                           float half, int& kbyte, float& f, float& wt) {
  const double dx = o[0] + n.DX;
  const double dy = o[1] + n.DY;
  double R2 = dx * dx + dy * dy;
  if (ND == 3) {
    const double dz = o[2] + n.DZ;
    R2 = R2 + dz * dz;
  }
  R2 = fmax(R2, rmin2);
  // R from the hardware reciprocal square root and one Newton step (relative
  // error ~1e-14, far below what the delay's fraction needs); the weight,
  // an FP32 value, from the FP32 one, as in the far pairs' arithmetic
  const double y0 = __builtin_amdgcn_rsq(R2);
  const double hy = 0.5 * R2 * y0;
  const double y1 = fma(y0, fma(-hy, y0, 0.5), y0);
  const double R = R2 > 0.0 ? R2 * y1 : 0.0;   // (a pixel on the sensor with r_min = 0: R = 0, an infinite weight)
  double d = R - n.KR;
  if (FRAC) d = d - t0fd;
  const double fl = floor(d);
  f = (float)(d - fl);
  wt = half * __builtin_amdgcn_rsqf((float)R2);
  kbyte = (int)fl * ESZ + base;
}

template <int ND, bool FRAC, int ESZ, bool CLAMP = true>
__device__ __forceinline__ void phase(const SC64& c, const Pix64& px, float, float, int& kbyte, double& f,
                                      double& wt) {
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
  kbyte = (int)fl * ESZ + c.BASE;
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

// Element k of a trace of n elements at base, read through a buffer resource
// whose range is the trace: the hardware's range check returns zero for any k
// outside 0..n-1 (a negative k is an offset beyond the range as an unsigned
// byte offset) without touching memory, so the caller needs no index test and
// no clamped address.  n * sizeof(T) < 2^31 (the planner caps traces at 2^22
// samples); n = 0 reads zeros.  Two calls at adjacent indices must not be
// merged into one wider load: its range check returns zero for element 0
// when the wider load starts at k = -1.
template <typename T>
__device__ __forceinline__ T trace_load(const T* base, int n, int k) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, n * (int)sizeof(T), 0x00020000);
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, k * 4, 0, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, k * 8, 0, 0));
  }
}

// Stores v as element k of a row of n elements at base, through a buffer
// resource whose range is the row: the hardware's range check drops stores
// with k outside 0..n-1, so the caller needs no lane test.
template <typename T>
__device__ __forceinline__ void row_store(T* base, int n, int k, T v) {
  static_assert(sizeof(T) == 4, "32-bit elements");
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, n * 4, 0x00020000);
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, k * 4, 0, 0);
}

// Non-finite test on a value's bits.  The operator kernels are built without
// NaN semantics, so a floating-point test, or a bit test the compiler
// recognises as one, may be folded away for a value it takes to be finite;
// the empty asm makes the bits opaque, so the test stays an integer test.
__device__ __forceinline__ bool non_finite_bits(float v) {
  unsigned b = __float_as_uint(v);
  asm volatile("" : "+v"(b));
  return (b & 0x7f800000u) == 0x7f800000u;
}
__device__ __forceinline__ bool non_finite_bits(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  asm volatile("" : "+v"(b));
  return (b & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
}

// floor(v + 0.5) as an int (round half up; the two taps of a pair are rounded
// the same way, so they still sum to the rounded total).  Under the operator
// files' build flags (no IEEE mode, no NaNs) this is one v_cvt_rpi_i32_f32,
// which the scheduler can move like any other instruction.
__device__ __forceinline__ int round_i(float v) {
  return (int)__builtin_floorf(v + 0.5f);
}

// Wave priority from progress q = 0, 1, 2, 3 (quarters of a work-group's main
// loop done): 3, 2, 1, 0.  The instruction arbiter favours the oldest waves,
// so without this the work-groups sharing a CU (the whole grid is one round)
// run their loops one after another and the last one finishes alone, with
// one wave per SIMD left to issue; lowering a wave's priority as it gets
// ahead keeps the CU's work-groups level and its VALU busy to the end.
__device__ __forceinline__ void progress_prio(int q) {
  if (q <= 0) __builtin_amdgcn_s_setprio(3);
  else if (q == 1) __builtin_amdgcn_s_setprio(2);
  else if (q == 2) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// Sum over the 64 lanes of a wave with DPP moves (no LDS round trips), in a
// fixed order; every lane gets the total.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]: every lane holds its quad's sum
  v += dpp_mov<0x124>(v);  // row_ror:4
  v += dpp_mov<0x128>(v);  // row_ror:8: every lane holds its row's sum
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

template <typename PH> constexpr size_t near_bytes() { return sizeof(PH) == 4 ? sizeof(Near32) : 0; }

__device__ __forceinline__ bool is_near(const OpParams& P, const double ref[3], const double sp[3]) {
  const double dx = ref[0] - sp[0], dy = ref[1] - sp[1], dz = ref[2] - sp[2];
  return dx * dx + dy * dy + dz * dz < P.near_r2;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// A^T: one work-group per base tile, one pixel per lane.  Sensors are taken in
// chunks: the chunk's per-sensor constants and each sensor's trace window
// (the samples any pixel of the tile can reach, zero outside 0..K-1) are
// staged in LDS, then every lane gathers its two taps per sensor from LDS.
// Within a chunk the sensors are ordered far-first (a deterministic
// compaction), so the fast FP32 loop runs without per-sensor tests and the
// few near sensors follow in an FP64-delay loop.
// With CG the epilogue also performs x += alpha p, s = A^T r - lambda x and the
// FP64 partial sums of ||s||^2 and ||x||^2.
template <typename T, typename PH, int ND, bool FRAC, bool CG>
__device__ __forceinline__ void bp_body(const OpParams& P, int tile, int pidx, const T* __restrict__ y,
                                        T* __restrict__ out, T* __restrict__ xcg, const T* __restrict__ pcg,
                                        const double* __restrict__ alpha, double lambda,
                                        double* __restrict__ part_s, double* __restrict__ part_x) {
  using SC = typename SCOf<PH>::type;
  using PX = typename PixOf<PH>::type;
  constexpr int TX = Tile<ND>::X, TY = Tile<ND>::Y, TZ = Tile<ND>::Z;
  constexpr bool F32 = sizeof(PH) == 4;  // FP32 delay arithmetic (with the FP64 near path)
  extern __shared__ __align__(16) unsigned char smem[];
  // window entries are (y_k, y_{k+1} - y_k) pairs: one LDS read gives a
  // pair's two taps' interpolation operands
  using T2 = T __attribute__((ext_vector_type(2)));
  constexpr int ESZ = (int)sizeof(T2);
  const BpLayout L = bp_layout(P.sc, P.wp, sizeof(T2), sizeof(SC), near_bytes<PH>());
  SC* sct = reinterpret_cast<SC*>(smem + L.sct);
  int* klo_s = reinterpret_cast<int*>(smem + L.klo);
  int* sid = reinterpret_cast<int*>(smem + L.sid);
  Near32* ntab = reinterpret_cast<Near32*>(smem + L.nd);
  T2* win = reinterpret_cast<T2*>(smem + L.win);
  __shared__ double red[4];
  __shared__ int cnt[8];

  const int bx = tile % P.ntile[0];
  const int by = (tile / P.ntile[0]) % P.ntile[1];
  const int bz = tile / (P.ntile[0] * P.ntile[1]);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
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
  const unsigned long long lt_mask = (1ull << lane) - 1ull;

  T acc = 0;
  for (int s0 = 0; s0 < P.S; s0 += P.sc) {
    progress_prio((4 * s0) / P.S);
    const int nsc = min(P.sc, P.S - s0);
    const bool mine = tid < nsc;
    double sp[3] = {0.0, 0.0, 0.0};
    bool in_trace = false, near = false;
    int kl = 0;
    if (mine) {
      sensor_pos<ND>(P, s0 + tid, sp);
      kl = window_lo<ND>(P, lo, hi, sp, &in_trace, P.wp);
      near = F32 && in_trace && is_near(P, ref, sp);
    }
    // far sensors first, then near ones; order within each group = sensor order
    const unsigned long long bfar = __ballot(mine && !near);
    const unsigned long long bnear = __ballot(mine && near);
    if (lane == 0) {
      cnt[wave] = __popcll(bfar);
      cnt[4 + wave] = __popcll(bnear);
    }
    __syncthreads();
    const int nfar = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    int far_before = 0, near_before = 0;
    for (int w = 0; w < wave; ++w) {
      far_before += cnt[w];
      near_before += cnt[4 + w];
    }
    if (mine) {
      const int pos = near ? nfar + near_before + __popcll(bnear & lt_mask) : far_before + __popcll(bfar & lt_mask);
      SC c;
      make_sc<ND>(P, ref, sp, kl, pos * P.wp, ESZ, in_trace, c);
      c.BASE += (int)(size_t)win;  // absolute LDS byte address of the row's reference sample
      sct[pos] = c;
      klo_s[pos] = in_trace ? kl : P.K + 8;  // inactive rows stage zeros
      sid[pos] = s0 + tid;
      if (near) {
        Near32 n;
        n.DX = ref[0] - sp[0];
        n.DY = ref[1] - sp[1];
        n.DZ = ref[2] - sp[2];
        n.KR = rint(sqrt(n.DX * n.DX + n.DY * n.DY + n.DZ * n.DZ));
        ntab[pos] = n;
      }
    }
    __syncthreads();
    // Stage the windows: wave w copies rows w, w+4, ... (row parameters are
    // wave-uniform, held in scalar registers), 64 entries of a row per step,
    // with the loads of eight rows in flight before their stores.  Each row
    // reads its sensor's trace through a buffer resource: samples outside
    // 0..K-1 and rows beyond the chunk (an empty range) read as zero.  Entry
    // i holds sample k = klo + i and the difference to sample k + 1.
    constexpr int RB = 8;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    for (int i0 = 0; i0 < P.wp; i0 += 64) {
      const int i = i0 + lane;
      for (int j0 = wv; j0 < nsc; j0 += 4 * RB) {
        T v0[RB], v1[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int j = j0 + 4 * u;
          const int jj = j < nsc ? j : 0;
          const int kl = __builtin_amdgcn_readfirstlane(klo_s[jj]);
          const int sj = __builtin_amdgcn_readfirstlane(sid[jj]);
          const T* tr = y + (size_t)sj * P.K;
          const int n = j < nsc ? P.K : 0;
          // Two loads, kept apart: merged into one two-element load, the
          // range check of a window starting before sample 0 also zeroes
          // sample 0 at k = -1 (measured), so the compiler must not see that
          // the second index is the first plus one.
          int k1 = kl + i + 1;
          asm volatile("" : "+v"(k1));
          v0[u] = trace_load(tr, n, kl + i);
          v1[u] = trace_load(tr, n, k1);
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int j = j0 + 4 * u;
          if (j < nsc && i < P.wp) {
            T2 e;
            e.x = v0[u];
            e.y = v1[u] - v0[u];
            win[j * P.wp + i] = e;
          }
        }
      }
    }
    __syncthreads();
    // Sensors whose arrivals miss the trace carry a finite weight and a
    // bounded delay into a zero row, so the loop needs no per-sensor test.
    // Only the FP64-delay kernels, where every sensor takes this loop, can
    // reach the distance clamp.
    constexpr bool CLAMP = !F32;
    // Four sensors per step: four delays, then four independent window
    // reads, then the sums in sensor order (the order never changes).
    int j = 0;
    for (; j + 4 <= nfar; j += 4) {
      int kb[4];
      PH f[4], w[4];
      T2 e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) phase<ND, FRAC, ESZ, CLAMP>(sct[j + u], px, t0f, P.hs2h, kb[u], f[u], w[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) e[u] = lds_load(reinterpret_cast<const T2*>(static_cast<size_t>(kb[u])));
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma((T)w[u], fma((T)f[u], e[u].y, e[u].x), acc);
    }
    for (; j < nfar; ++j) {
      int kb;
      PH f, w;
      phase<ND, FRAC, ESZ, CLAMP>(sct[j], px, t0f, P.hs2h, kb, f, w);
      const T2 e = lds_load(reinterpret_cast<const T2*>(static_cast<size_t>(kb)));
      acc = fma((T)w, fma((T)f, e.y, e.x), acc);
    }
    if constexpr (F32) {
      if (nfar < nsc) {
        double o[3];
        pix_offsets<ND>(P, lx, ly, lz, o);
        for (; j < nsc; ++j) {
          const SC32& c = sct[j];
          int kb;
          float f, w;
          phase_near<ND, FRAC, ESZ>(ntab[j], o, P.rmin * P.rmin, P.t0fd, c.BASE, 1.0f, kb, f, w);
          const T2 e = lds_load(reinterpret_cast<const T2*>(static_cast<size_t>(kb)));
          acc = fma((T)w, fma((T)f, e.y, e.x), acc);
        }
      }
    }
    __syncthreads();
  }

  const size_t idx = ((size_t)iz * P.ny + iy) * P.nx + ix;
  const T scale = (T)P.out_scale;   // (sums of w y)
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
    part_s[pidx] = ss;
    part_x[pidx] = xx;
  }
}

// ---------------------------------------------------------------------------
// A: one work-group per (sensor s, segment of fseg samples of its trace), one
// pixel per lane and four pixels per lane per base tile.  The work-group owns
// its outputs, so no partial rows leave it and no other work-group adds into
// them.
//
// Rounds of kFwdList base tiles: every lane tests one tile's window against
// the segment (plus a window's margin, since a tile reaching the segment may
// also reach its neighbours) and the tiles that reach it are compacted into
// an LDS list, in tile order, with their per-(tile, sensor) constants.  Wave w
// then takes groups of G consecutive list entries, groups w, w+4, ...:
// the sensor and tiles are uniform across the wave, so the delay constants
// are wave-uniform LDS reads, and each lane keeps its four pixels' offsets
// from a tile centre in registers for the whole kernel.  The next group's x
// values are loaded while the current group is processed.
//
// Bins, FP32 delay arithmetic (PA_F32, PA_MIXED), by default: the taps of a
// group go to a wave-private row of 32-bit fixed-point bins (LDS integer adds
// are fast on gfx950 and their sums do not depend on order), scaled by
// 2^30 / B with B = sum over the group's tiles of (sum of |x| over the tile)
// / (2 dmin), a bound on every partial sum of a bin; the touched part of the
// row is then added, in FP64, into the wave's histogram and cleared.
// Otherwise (PA_F64, or FP64 bins chosen for FP32 delay arithmetic) taps go
// straight into the wave's FP64 histogram with LDS FP64 adds.  Either way
// each wave adds its tiles in list order and the four waves' histograms are
// summed in a fixed order, so y is the same on every run.
// A non-finite x in a group makes its bound non-finite (fixed-point rows) or
// its taps non-finite (FP64 bins), so non-finite inputs give non-finite traces.
template <typename T, typename PH, int ND, bool FRAC, bool FIX>
__device__ __forceinline__ void fp_body(const OpParams& P, int b, int pidx, const T* __restrict__ x,
                                        T* __restrict__ y, double* __restrict__ part_q) {
  using SCA = typename SCOf<PH>::type;    // the adjoint's constants, made by the same function
  using SC = typename std::conditional<sizeof(PH) == 4, FpSC32, SC64>::type;
  using PX = typename PixOf<PH>::type;
  constexpr int TX = Tile<ND>::X, TY = Tile<ND>::Y, TZ = Tile<ND>::Z;
  constexpr int PPL = TX * TY * TZ / 64;   // pixels per lane per base tile
  constexpr int G = kFwdGroupMax / 2;
  constexpr bool P32 = sizeof(PH) == 4;
  constexpr int HB = FIX ? 4 : 8;          // bytes per bin of the rows the taps go to
  static_assert(P32 || !FIX, "fixed-point rows are for FP32 delay arithmetic");
  extern __shared__ __align__(16) unsigned char smem[];
  const FpLayout L = fp_layout(P.fbins, P.wp, sizeof(SC), FIX);
  SC* lst = reinterpret_cast<SC*>(smem + L.lst);
  FpTile* ltab = reinterpret_cast<FpTile*>(smem + L.ltab);
  __shared__ double red[4];
  __shared__ int cnt[4], ccnt[4];
  __shared__ int ctile[kFwdList];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int s = b / P.fnseg;
  const int k0 = (b - s * P.fnseg) * P.fseg;   // first sample of this work-group's segment
  const int hlo = k0 - P.wp - 1;               // sample of histogram bin 0
  double* hist = reinterpret_cast<double*>(smem + L.hist) + wave * P.fbins;
  int* irow = reinterpret_cast<int*>(smem + L.irow + (size_t)wave * align16((size_t)P.fbins * 4));
  for (int e = lane; e < P.fbins; e += 64) {
    hist[e] = 0.0;
    if constexpr (FIX) irow[e] = 0;
  }
  const int rbase = FIX ? (int)(size_t)irow : (int)(size_t)hist;  // LDS byte address of this wave's tap row
  double sp[3];
  sensor_pos<ND>(P, s, sp);
  // FP32 copies for the candidate test: tile-centre grid, sensor, t0 and the
  // base tile's half-diagonal plus a margin for FP32 rounding (sample units)
  float fc_org[3], fc_step[3], fsp[3];
  {
    const int T3[3] = {TX, TY, TZ};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      fc_org[a] = (float)(P.org[a] + 0.5 * (T3[a] - 1) * P.hs);
      fc_step[a] = (float)(T3[a] * P.hs);
      fsp[a] = (float)sp[a];
    }
  }
  const float fT0 = (float)((double)P.t0i + P.t0fd);
  const float f_hd = (float)(0.5 * P.hs * sqrt((double)((TX - 1) * (TX - 1) + (TY - 1) * (TY - 1) + (TZ - 1) * (TZ - 1)))) + 2.f;
  // this lane's pixels of a base tile: p = lane + 64 q
  PX px[PPL];
  int poff[PPL], plim[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    const int p = lane + 64 * q;
    const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
    make_pix<ND>(P, lx, ly, lz, px[q]);
    poff[q] = (lz * P.ny + ly) * P.nx + lx;
    plim[q] = lx | ly << 8 | lz << 16;
  }
  const float t0f = P.t0f;
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  constexpr int kFull = TX | TY << 8 | TZ << 16;  // FpTile::lim of a tile inside the image

  for (int c0 = 0; c0 < P.n_tiles; c0 += kFwdList) {
    // ---- list the tiles of this round whose window reaches the segment.
    // A cheap FP32 test on the tile centre's distance first (a superset of
    // the tiles that reach the segment), then the exact FP64 window only for
    // the candidates, compacted onto the first lanes.
    int t = c0 + tid;
    bool cand = false;
    if (t < P.n_tiles) {
      const int cx = t % P.ntile[0];
      const int cy = (t / P.ntile[0]) % P.ntile[1];
      const int cz = t / (P.ntile[0] * P.ntile[1]);
      const float dx = fc_org[0] + (float)cx * fc_step[0] - fsp[0];
      const float dy = fc_org[1] + (float)cy * fc_step[1] - fsp[1];
      const float dz = ND == 3 ? fc_org[2] + (float)cz * fc_step[2] - fsp[2] : 0.f;
      const float dc = __builtin_sqrtf(dx * dx + dy * dy + dz * dz) - fT0;
      cand = dc - f_hd < (float)(k0 + P.fseg + 4) && dc + (float)P.wp > (float)(k0 - 4);
    }
    {
      const unsigned long long cb = __ballot(cand);
      __syncthreads();  // the previous round's list and candidates have been consumed
      if (lane == 0) ccnt[wave] = __popcll(cb);
      __syncthreads();
      int cbefore = 0;
      for (int w = 0; w < wave; ++w) cbefore += ccnt[w];
      if (cand) ctile[cbefore + __popcll(cb & lt_mask)] = t;
      __syncthreads();
    }
    const int nc = ccnt[0] + ccnt[1] + ccnt[2] + ccnt[3];
    t = tid < nc ? ctile[tid] : P.n_tiles;
    bool take = false;
    int kl = 0;
    double ref[3], dmin = 0.0;
    int bx = 0, by = 0, bz = 0;
    if (t < P.n_tiles) {
      bx = t % P.ntile[0];
      by = (t / P.ntile[0]) % P.ntile[1];
      bz = t / (P.ntile[0] * P.ntile[1]);
      tile_ref<ND>(P, bx, by, bz, ref);
      double lo[3], hi[3];
      const int T3[3] = {TX, TY, TZ};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double half = 0.5 * (T3[a] - 1) * P.hs;
        lo[a] = ref[a] - half;
        hi[a] = ref[a] + half;
      }
      bool in_trace = false;
      kl = window_lo<ND>(P, lo, hi, sp, &in_trace, P.wp, &dmin);
      take = in_trace && kl < k0 + P.fseg && kl + P.wp > k0;
    }
    const unsigned long long bal = __ballot(take);
    if (lane == 0) cnt[wave] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += cnt[w];
    const int nl = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    if (take) {
      const int pos = before + __popcll(bal & lt_mask);
      SCA c;
      make_sc<ND>(P, ref, sp, hlo, 0, HB, true, c);  // tap bins relative to the histogram
      lst[pos] = fp_sc(c);
      FpTile ft;
      ft.off = kl - hlo;
      ft.xoff = ((bz * TZ) * P.ny + by * TY) * P.nx + bx * TX;
      ft.lim = min(TX, P.nx - bx * TX) | min(TY, P.ny - by * TY) << 8 | min(TZ, P.nz - bz * TZ) << 16 |
               ((P32 && is_near(P, ref, sp)) ? kFpNear : 0);
      ft.ib = (float)(0.5 / dmin);
      ltab[pos] = ft;
    }
    if (tid >= nl && tid < (nl + kFwdGroupMax - 1) / kFwdGroupMax * kFwdGroupMax) {  // pad the list to whole groups
      FpTile ft;
      ft.off = 0;
      ft.xoff = 0;
      ft.lim = 0;
      ft.ib = 0.f;
      ltab[tid] = ft;
    }
    __syncthreads();

    // ---- scatter: wave w takes groups w, w+4, ... of G consecutive entries
    const int ngroups = (nl + G - 1) / G;
    T xn[G][PPL];
    // (the list is padded to whole groups with entries of no pixels, lim = 0,
    // so the loads need no bounds test on the list; partial tiles load their
    // first pixel in place of pixels outside the image and zero it)
    auto load_x = [&](int g0, T (&xv)[G][PPL]) {
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int j = g0 * G + u;
        const int xoff = __builtin_amdgcn_readfirstlane(ltab[j].xoff);
        const int lim = __builtin_amdgcn_readfirstlane(ltab[j].lim) & (kFpNear - 1);
        const T* __restrict__ xb = x + xoff;   // wave-uniform base, per-lane 32-bit offsets
        if (lim == kFull) {
#pragma unroll
          for (int q = 0; q < PPL; ++q) xv[u][q] = xb[(unsigned)poff[q]];
        } else {
#pragma unroll
          for (int q = 0; q < PPL; ++q) {
            const bool in = (plim[q] & 0xff) < (lim & 0xff) && ((plim[q] >> 8) & 0xff) < ((lim >> 8) & 0xff) &&
                            (plim[q] >> 16) < (lim >> 16);
            const T v = xb[in ? (unsigned)poff[q] : 0u];
            xv[u][q] = in ? v : (T)0;
          }
        }
      }
    };
    if (wave < ngroups) load_x(wave, xn);
    for (int gi = wave; gi < ngroups; gi += 4) {
      T xv[G][PPL];
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int q = 0; q < PPL; ++q) xv[u][q] = xn[u][q];
      if (gi + 4 < ngroups) load_x(gi + 4, xn);
      const int j0 = gi * G;
      const int nu = min(G, nl - j0);
      float scl = 0.f;
      double inv = 0.0;
      int rlo = 0, rhi = 0;   // bins of the int row this group touches
      if constexpr (FIX) {
        // the group's bound and fixed-point scale
        float sa = 0.f;
        rlo = P.fbins;
#pragma unroll
        for (int u = 0; u < G; ++u) {
          if (u < nu) {
            const float ib = ltab[j0 + u].ib;
            const int off = __builtin_amdgcn_readfirstlane(ltab[j0 + u].off);
            float su = 0.f;
#pragma unroll
            for (int q = 0; q < PPL; ++q) su += fabsf((float)xv[u][q]);
            sa = fmaf(su, ib, sa);
            rlo = min(rlo, off);
            rhi = max(rhi, off + P.wp);
          }
        }
        const float bound = wave_sum(sa) * (1.0f + 1.0f / 256.0f);
        // a NaN or infinite x (tested on the loaded values' bits), or a bound
        // beyond float: the group's windows become NaN
        bool nf = non_finite_bits(bound);
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
          for (int q = 0; q < PPL; ++q) nf |= non_finite_bits(xv[u][q]);
        if (__ballot(nf) != 0) {
          for (int e = rlo + lane; e < rhi; e += 64)   // stored as bits, out of reach of NaN folding
            reinterpret_cast<long long*>(hist)[e] = 0x7ff8000000000000ll;
          continue;
        }
        if (bound == 0.0f) continue;  // all-zero tiles: nothing to add
        float b = bound;
        double post = 1.0;
        if (b < 0x1p-60f) {
          // tiny x (below ~1e-18): scale the group's values by an exact power
          // of two first, so 2^30 / bound stays finite and the fixed point
          // keeps its full range; the rows are scaled back on the way out
          const int e = min(120, -ilogbf(b));
          const float sx = ldexpf(1.0f, e);
#pragma unroll
          for (int u = 0; u < G; ++u)
#pragma unroll
            for (int q = 0; q < PPL; ++q) xv[u][q] = xv[u][q] * (T)sx;
          b *= sx;
          post = ldexp(1.0, -e);
        }
        // the bound is of taps w x / 2: the fixed point takes 2^30 / b times
        // that, so w x is scaled by half of it and each integer read back
        // at twice 1 / scale
        scl = 1073741824.0f * __builtin_amdgcn_rcpf(b);
        inv = post / (double)scl;
        scl *= 0.5f;
        inv *= 2.0;
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        if (u >= nu) break;
        SC c = lst[j0 + u];
        c.BASE += rbase;
        const int near = __builtin_amdgcn_readfirstlane(ltab[j0 + u].lim) & kFpNear;
        if (!P32 || near == 0) {
#pragma unroll
          for (int q = 0; q < PPL; ++q) {
            int kb;
            PH f, wt;
            if constexpr (FIX) {
              phase<ND, FRAC, HB, false>(c, px[q], t0f, P.hs2h, kb, f, wt);
              const float vs = (wt * (float)xv[u][q]) * scl;
              const int it = round_i(vs);
              const int i1 = round_i(vs * f);
              int* bin = reinterpret_cast<int*>(static_cast<size_t>(kb));
              lds_add(bin, it - i1);
              lds_add(bin + 1, i1);
            } else {
              phase<ND, FRAC, HB, false>(c, px[q], t0f, P.hs2h, kb, f, wt);
              const double v = (double)wt * (double)xv[u][q];
              const double a1 = v * (double)f;
              double* bin = reinterpret_cast<double*>(static_cast<size_t>(kb));
              lds_add(bin, v - a1);
              lds_add(bin + 1, a1);
            }
          }
        } else if constexpr (P32) {
          // sensor among or near the tile's pixels: delays from FP64 coordinates
          const int xo = ltab[j0 + u].xoff;
          const int pl = P.nx * P.ny;
          double rf[3];
          tile_ref<ND>(P, (xo % P.nx) / TX, ((xo % pl) / P.nx) / TY, (xo / pl) / TZ, rf);
          Near32 nn;
          nn.DX = rf[0] - sp[0];
          nn.DY = rf[1] - sp[1];
          nn.DZ = rf[2] - sp[2];
          nn.KR = rint(sqrt(nn.DX * nn.DX + nn.DY * nn.DY + nn.DZ * nn.DZ));
          const double rmin2 = P.rmin * P.rmin;
#pragma unroll
          for (int q = 0; q < PPL; ++q) {
            const int p = lane + 64 * q;
            double o[3];
            pix_offsets<ND>(P, p % TX, (p / TX) % TY, p / (TX * TY), o);
            int kb;
            float f, wt;
            phase_near<ND, FRAC, HB>(nn, o, rmin2, P.t0fd, c.BASE, 1.0f, kb, f, wt);
            if constexpr (FIX) {
              const float vs = (wt * (float)xv[u][q]) * scl;
              const int it = round_i(vs);
              const int i1 = round_i(vs * f);
              int* bin = reinterpret_cast<int*>(static_cast<size_t>(kb));
              lds_add(bin, it - i1);
              lds_add(bin + 1, i1);
            } else {
              const double v = (double)wt * (double)xv[u][q];
              const double a1 = v * (double)f;
              double* bin = reinterpret_cast<double*>(static_cast<size_t>(kb));
              lds_add(bin, v - a1);
              lds_add(bin + 1, a1);
            }
          }
        }
      }
      if constexpr (FIX) {
        // the touched bins into the histogram (this wave's own bins: plain LDS
        // reads and writes, each lane its own), then cleared for the next group
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int e = rlo + lane; e < rhi; e += 64) {
          const int v = irow[e];
          if (v != 0) {
            hist[e] += (double)v * inv;
            irow[e] = 0;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
  __syncthreads();

  // ---- the segment out: the four waves' histograms in a fixed order
  const double* h0 = reinterpret_cast<const double*>(smem + L.hist);
  const double scale = P.out_scale;   // (sums of w x)
  const int kn = min(P.fseg, P.K - k0);
  double qq = 0.0;
  for (int i = tid; i < kn; i += kBlock) {
    const int e = i + P.wp + 1;
    const double v = (h0[e] + h0[P.fbins + e]) + (h0[2 * P.fbins + e] + h0[3 * P.fbins + e]);
    const T out = (T)(v * scale);
    y[(size_t)s * P.K + k0 + i] = out;
    qq += (double)out * (double)out;
  }
  if (part_q) {
    qq = block_sum(qq, red);
    if (tid == 0) part_q[pidx] = qq;
  }
}

// ---------------------------------------------------------------------------
// A through partial rows (PA_F32 with a workspace), pass 1: one work-group
// per (forward tile, chunk of 64 sensors); lane =
// sensor, wave w walks base tiles w, w+4, ... of the forward tile (or, with
// fewer than four base tiles, a quarter or half of one) one pixel at a time
// (the pixel is uniform across the wave).  Each lane scatters its two
// taps into its own sensor's LDS histogram row, so the lanes of one ds_add
// never collide on an address.  The rows are then written out with plain
// coalesced stores, with the first sample of each row in a table.
template <int ND, bool FRAC, bool CG>
__device__ __forceinline__ void fp2_body(const OpParams& P, int b, const float* __restrict__ x, float* __restrict__ rows,
                                         int* __restrict__ klo_tab, const CgDirArgs& cg) {
  using T = float;
  using SC = SC32;
  using PX = Pix32;
  constexpr int TX = Tile<ND>::X, TY = Tile<ND>::Y, TZ = Tile<ND>::Z;
  constexpr int NS = kSensorsPerFwdBlock;
  constexpr bool F32 = true;
  extern __shared__ __align__(16) unsigned char smem[];
  const Fp2Layout L = fp2_layout(P.wpa, P.nsub);
  // Histogram bins.  FP64 kernels add doubles.  FP32 kernels add 32-bit
  // fixed-point integers (LDS float adds are slow on gfx950, integer adds are
  // not): lane s scales its taps by 2^30 / B_s, where B_s bounds the sum of
  // |tap| over the whole forward tile, so no bin can overflow; integer sums
  // do not depend on their order, and each row is converted back once, when
  // it is written out.
  using H = typename std::conditional<F32, int, double>::type;
  constexpr int HB = (int)sizeof(H);
  H* hist = reinterpret_cast<H*>(smem + L.hist);
  T* xs = reinterpret_cast<T*>(smem + L.xs);
  int* klo_a = reinterpret_cast<int*>(smem + L.klo);
  double* inv_a = reinterpret_cast<double*>(smem + L.inv);
  __shared__ double red[4];
  __shared__ double ppw[4];   // per-wave sums of p_k^2 (direction update)

  // chunk-major: with the XCD remap of the launch, each XCD takes a
  // contiguous run of (chunk, tile) blocks, so one chunk's rows are written
  // within two XCDs, where pass 2 (remapped the same way) reads them
  // (b, chunk and at are uniform; saying so keeps the row addresses scalar)
  const int chunk = __builtin_amdgcn_readfirstlane(b / P.n_atiles);
  const int at = __builtin_amdgcn_readfirstlane(b - chunk * P.n_atiles);
  const int ax = at % P.natile[0];
  const int ay = (at / P.natile[0]) % P.natile[1];
  const int az = at / (P.natile[0] * P.natile[1]);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
  const int s = chunk * NS + lane;
  const bool s_ok = s < P.S;

  // this lane's sensor (its load goes out with the x loads below)
  double sp[3];
  sensor_pos<ND>(P, s_ok ? s : P.S - 1, sp);
  double* sa_m = reinterpret_cast<double*>(smem + L.inv) + NS;  // [nsub][4] per-wave sums of |x|
  // The forward tile's x values, staged in LDS, and each wave's sum of |x|
  // over its 64 pixels of every base tile.  Base tiles go in groups of four:
  // a group's global loads are all issued before the first is used, and its
  // four wave sums share the shuffle steps.  With the CGLS direction update
  // the staged values are p_k = s_k + beta p_{k-1} (the first two groups'
  // loads of s and p go out before beta is formed), the first sensor chunk
  // writes them out, and each thread sums its p_k^2.
  bool nfx = false;   // a NaN or infinite x among this lane's staged values
  double pp = 0.0;
  {
    constexpr int MG = 4, NB = 2 * MG;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    // element index of this thread's pixel of base tile m, -1 outside the image
    auto pix_index = [&](int m) -> int64_t {
      const int bx = ax * P.msub[0] + m % P.msub[0];
      const int by = ay * P.msub[1] + (m / P.msub[0]) % P.msub[1];
      const int bz = az * P.msub[2] + m / (P.msub[0] * P.msub[1]);
      const int ix = bx * TX + lx, iy = by * TY + ly, iz = bz * TZ + lz;
      return m < P.nsub && ix < P.nx && iy < P.ny && iz < P.nz ? ((int64_t)iz * P.ny + iy) * P.nx + ix : -1;
    };
    auto stage = [&](int m0, const T (&v)[MG]) {
      double a[MG];
#pragma unroll
      for (int u = 0; u < MG; ++u) {
        nfx |= non_finite_bits(v[u]);
        if (m0 + u < P.nsub) xs[(m0 + u) * kBlock + tid] = v[u];
        a[u] = fabs((double)v[u]);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int u = 0; u < MG; ++u) a[u] += __shfl_xor(a[u], o, 64);
      if (lane == 0) {
#pragma unroll
        for (int u = 0; u < MG; ++u)
          if (m0 + u < P.nsub) sa_m[(m0 + u) * 4 + wave] = a[u];
      }
    };
    if constexpr (CG) {
      const bool rp = cg.k >= 1;   // p_{k-1} is read
      // the scalars beta needs go out first, with the vector loads below
      const int st_k = *cg.status;
      const double gold = cg.gamma[rp ? cg.k - 1 : 0];
      int64_t ib[NB];
      T sv[NB], pv[NB];
#pragma unroll
      for (int m = 0; m < NB; ++m) {
        ib[m] = pix_index(m);
        // (unconditional loads, element 0 for pixels outside: they go out
        // back to back, and dirv() drops the extra values)
        sv[m] = cg.s[ib[m] >= 0 ? ib[m] : 0];
        pv[m] = cg.p_old[ib[m] >= 0 ? ib[m] : 0];   // (read also for k = 0: beta is 0 then)
      }
      // beta = ||s_k||^2 / gamma[k - 1]: the same sum, in the same order, in
      // every work-group
      const double ss = dev::sum_partials(cg.part_s, cg.gs, red);
      double beta = 0.0;
      if (rp) beta = (st_k >= 0 || !(gold > 0.0)) ? 0.0 : ss / gold;
      if (blockIdx.x == 0) {   // gamma[k] and history row k, once
        const double xx = dev::sum_partials(cg.part_x, cg.gx, red);
        const double rr = dev::sum_partials(cg.part_r, cg.gr, red);
        if (tid == 0) {
          cg.gamma[cg.k] = ss;
          if (cg.hist) {
            cg.hist[3 * cg.k + 0] = sqrt(rr);
            cg.hist[3 * cg.k + 1] = sqrt(ss);
            cg.hist[3 * cg.k + 2] = rr + cg.lambda * xx;
          }
        }
      }
      auto dirv = [&](int64_t i, T sk, T pk) -> T {
        if (i < 0) return (T)0;
        const T t = (T)((double)sk + (beta != 0.0 ? beta * (double)pk : 0.0));
        if (chunk == 0) cg.p_new[i] = t;
        pp += (double)t * (double)t;
        return t;
      };
#pragma unroll
      for (int g = 0; g < NB / MG; ++g) {
        if (g * MG < P.nsub) {
          T v[MG];
#pragma unroll
          for (int u = 0; u < MG; ++u) v[u] = dirv(ib[g * MG + u], sv[g * MG + u], pv[g * MG + u]);
          stage(g * MG, v);
        }
      }
      for (int m0 = NB; m0 < P.nsub; m0 += MG) {
        int64_t i2[MG];
        T s2[MG], p2[MG], v[MG];
#pragma unroll
        for (int u = 0; u < MG; ++u) {
          i2[u] = pix_index(m0 + u);
          s2[u] = cg.s[i2[u] >= 0 ? i2[u] : 0];
          p2[u] = cg.p_old[i2[u] >= 0 ? i2[u] : 0];
        }
#pragma unroll
        for (int u = 0; u < MG; ++u) v[u] = dirv(i2[u], s2[u], p2[u]);
        stage(m0, v);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) pp += __shfl_xor(pp, o, 64);
      if (lane == 0) ppw[wave] = pp;
    } else {
      for (int m0 = 0; m0 < P.nsub; m0 += MG) {
        T v[MG];
#pragma unroll
        for (int u = 0; u < MG; ++u) {
          const int64_t i = pix_index(m0 + u);
          v[u] = i >= 0 ? x[i] : (T)0;
        }
        stage(m0, v);
      }
    }
  }
  // Fixed-point scale: a tap of pixel p in base tile m is at most
  // |x_p| / (2 dmin_m), dmin_m being the distance from this lane's sensor to
  // base tile m (clamped at r_min), so B_s = sum_m (sum_{p in m} |x_p|) /
  // (2 dmin_m) bounds every partial sum of the row.  The four waves hold the
  // same 64 sensors, so the FP64 per-sensor work is split between them: wave
  // w forms the terms of base tiles w, w + 4, ..., wave 0 the window over the
  // forward tile, and wave 0 adds the terms in tile order.
  double* bterm = sa_m + 4 * P.nsub;                              // [nsub][64] bound terms
  float* scl_a = reinterpret_cast<float*>(bterm + P.nsub * NS);   // [64] fixed-point scales
  const bool tile_nf = __syncthreads_or(nfx) != 0;   // (also the barrier for sa_m and ppw)
  if constexpr (CG) {
    if (chunk == 0 && tid == 0) cg.part_p[at] = (ppw[0] + ppw[1]) + (ppw[2] + ppw[3]);
  }
  // Tiny x (the forward tile's sum below ~1e-18): scale the staged values
  // by an exact power of two, so 2^30 / B_s stays finite and the fixed
  // point keeps its full range; the rows are scaled back on the way out.
  // (The sum is the same in every lane, so the branch is uniform.)
  double tsum = 0.0;
  for (int m = 0; m < 4 * P.nsub; ++m) tsum += sa_m[m];
  double post = 1.0, pre = 1.0;
  if (!tile_nf && tsum > 0.0 && tsum < 0x1p-60) {
    const int e = min(120, -ilogb(tsum));
    const float sx = ldexpf(1.0f, e);
    for (int i = tid; i < P.nsub * kBlock; i += kBlock) xs[i] *= sx;
    pre = (double)sx;
    post = ldexp(1.0, -e);
  }
  for (int m = wave; m < P.nsub; m += 4) {
    const double sa = pre * ((sa_m[m * 4 + 0] + sa_m[m * 4 + 1]) + (sa_m[m * 4 + 2] + sa_m[m * 4 + 3]));
    double term = 0.0;
    if (sa != 0.0) {
      const int bx = ax * P.msub[0] + m % P.msub[0];
      const int by = ay * P.msub[1] + (m / P.msub[0]) % P.msub[1];
      const int bz = az * P.msub[2] + m / (P.msub[0] * P.msub[1]);
      double r0[3], lo[3], hi[3];
      tile_ref<ND>(P, bx, by, bz, r0);
      const int T3[3] = {TX, TY, TZ};
      double d2 = 0.0;
#pragma unroll
      for (int a = 0; a < ND; ++a) {
        lo[a] = r0[a] - 0.5 * (T3[a] - 1) * P.hs;
        hi[a] = r0[a] + 0.5 * (T3[a] - 1) * P.hs;
        const double e = fmax(fmax(lo[a] - sp[a], sp[a] - hi[a]), 0.0);
        d2 += e * e;
      }
      term = sa * (0.5 / fmax(sqrt(d2), P.rmin));
    }
    bterm[m * NS + lane] = term;
  }
  if (wave == 0) {
    // this lane's window over the whole forward tile
    bool in_trace;
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
    const int kl0 = window_lo<ND>(P, lo, hi, sp, &in_trace, P.wpa);
    klo_a[lane] = s_ok && in_trace ? kl0 : P.K + 8;
  }
  for (int e = tid; e < NS * P.wpa; e += kBlock) hist[e] = 0;
  __syncthreads();
  if (wave == 0) {
    double bound = 0.0;
    for (int m = 0; m < P.nsub; ++m) bound += bterm[m * NS + lane];
    bound *= 1.0 + 1.0 / 1024.0;
    // A NaN or infinite x in the forward tile (or a bound beyond double)
    // gives the rows a NaN scale, so their traces come out NaN, not zero.
    const bool bad = tile_nf || non_finite_bits(bound);
    float sc = 0.f;
    if (!bad && bound > 0.0 && bound < 1e300) sc = (float)(1073741824.0 / bound);
    scl_a[lane] = sc;
    // (selected as integer bits: under the no-NaN build flags a NaN operand
    // of a floating-point select may be folded away)
    const long long v = __double_as_longlong(sc > 0.f ? post / (double)sc : 0.0);
    reinterpret_cast<long long*>(inv_a)[lane] = bad ? 0x7ff8000000000000ll : v;
  }
  __syncthreads();
  const float scl = scl_a[lane];
  const int kl = klo_a[lane];
  const bool active = kl != P.K + 8;

  const float t0f = P.t0f;
  // Work items: (base tile m, part).  With fewer than four base tiles per
  // forward tile the waves split each tile's pixels into `parts` ranges.
  const int parts = P.nsub >= 4 ? 1 : 4 / P.nsub;
  for (int item = wave; item < P.nsub * parts; item += 4) {
    const int m = item / parts;
    const int part = item - m * parts;
    const int bx = ax * P.msub[0] + m % P.msub[0];
    const int by = ay * P.msub[1] + (m / P.msub[0]) % P.msub[1];
    const int bz = az * P.msub[2] + m / (P.msub[0] * P.msub[1]);
    const int nlx = __builtin_amdgcn_readfirstlane(min(TX, P.nx - bx * TX));
    const int nly = __builtin_amdgcn_readfirstlane(min(TY, P.ny - by * TY));
    const int nlz = __builtin_amdgcn_readfirstlane(min(TZ, P.nz - bz * TZ));
    if (nlx <= 0 || nly <= 0 || nlz <= 0) continue;
    double ref[3];
    tile_ref<ND>(P, bx, by, bz, ref);
    // Near (tile, sensor) pairs take benign constants and a zero scale here and
    // are added afterwards, one sensor at a time with one pixel per lane, so
    // the wave never runs the FP64 delay path for all of its pixels.
    const bool near = F32 && active && is_near(P, ref, sp);
    // a wave with near pairs of this tile to add after its loop keeps its
    // priority a quarter longer, so that work overlaps the other waves' loops
    const bool near_work = __ballot(near) != 0;
    SC c;
    make_sc<ND>(P, ref, sp, kl, lane * P.wpa, HB, active && !near, c);
    c.BASE += (int)(size_t)hist;  // absolute LDS byte address
    // w x times half the fixed-point scale (the bound is of taps w x / 2,
    // and the rows hold sums of w x / 2); near and inactive pairs add zeros here
    const float scl_m = active && !near ? 0.5f * scl : 0.f;
    asm volatile("" : "+v"(c.BASE));  // keep "k * HB + BASE" a single shift-add
    const T* xm = xs + m * kBlock;
    // Every pixel of the base tile, in order, four per step.  Pixels beyond
    // the image edge have x = 0 (and taps inside the window), so they add
    // zeros.  The pixel offsets come from the constant table by scalar loads
    // and the four x values from one LDS read, issued for the next four
    // pixels before this step's LDS adds (the last step reads four entries
    // past the range, into the arrays' slack); two register sets alternate.
    constexpr int NPIX = TX * TY * TZ;
    static_assert(NPIX % 32 == 0, "eight pixels per loop trip and up to four parts");
    const int p_lo = part * (NPIX / parts);
    const int p_hi = p_lo + NPIX / parts;
    const PX* ptab = pix_table<ND>();
    float hs2v = P.hs2h;
    asm volatile("" : "+v"(hs2v));  // a VGPR operand: the pixel's uq is the FMA's one scalar operand
    int po = p_lo;
    PX pa_[4], pb_[4];
    float4 xa_, xb_;
    auto load4 = [&](PX (&pp)[4], float4& xx) {
#pragma unroll
      for (int j = 0; j < 4; ++j) pp[j] = ptab[po + j];
      xx = *reinterpret_cast<const float4*>(xm + po);
      po += 4;
    };
    auto scatter4 = [&](const PX (&pp)[4], const float4& xx) {
      const float xv[4] = {xx.x, xx.y, xx.z, xx.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int kb;
        T f, wt;
        phase<ND, FRAC, HB, false>(c, pp[j], t0f, hs2v, kb, f, wt);
        H* bin = reinterpret_cast<H*>(static_cast<size_t>(kb));
        const float vs = (wt * xv[j]) * scl_m;
        const int i1 = round_i(vs * f);
        lds_add(bin, round_i(vs) - i1);
        lds_add(bin + 1, i1);
      }
    };
    load4(pa_, xa_);
    for (int p = p_lo; p < p_hi; p += 8) {
      if (((p - p_lo) & 63) == 0) progress_prio(((p - p_lo) * 4) / (p_hi - p_lo) - (near_work ? 1 : 0));
      load4(pb_, xb_);
      scatter4(pa_, xa_);
      load4(pa_, xa_);
      scatter4(pb_, xb_);
    }
    if constexpr (F32) {
      uint64_t nm = part == 0 ? __ballot(near) : 0;  // the near pairs of tile m, once
      if (nm != 0) {
        const double rmin2 = P.rmin * P.rmin;
        // this lane's row base for its own sensor, as the far constants would have it
        const double kr_l = rint(sqrt((ref[0] - sp[0]) * (ref[0] - sp[0]) + (ref[1] - sp[1]) * (ref[1] - sp[1]) +
                                      (ref[2] - sp[2]) * (ref[2] - sp[2])));
        const int base_l = ((int)kr_l - P.t0i - kl + lane * P.wpa) * HB + (int)(size_t)hist;
        while (nm != 0) {
          const int j = __builtin_ctzll(nm);
          nm &= nm - 1;
          Near32 nn;
          nn.DX = ref[0] - __shfl(sp[0], j);
          nn.DY = ref[1] - __shfl(sp[1], j);
          nn.DZ = ref[2] - __shfl(sp[2], j);
          nn.KR = __shfl(kr_l, j);
          const int base = __shfl(base_l, j);
          const float scl_j = __shfl(scl, j);
          for (int pix = lane; pix < TX * TY * TZ; pix += 64) {
            const int lx = pix % TX, ly = (pix / TX) % TY, lz = pix / (TX * TY);
            if (lx >= nlx || ly >= nly || lz >= nlz) continue;
            double o[3];
            pix_offsets<ND>(P, lx, ly, lz, o);
            int kb;
            float f, wt;
            phase_near<ND, FRAC, HB>(nn, o, rmin2, P.t0fd, base, 0.5f, kb, f, wt);
            const float vs = (wt * xm[pix]) * scl_j;
            const int it = (int)__builtin_rintf(vs);
            const int i1 = (int)__builtin_rintf(vs * f);
            H* bin = reinterpret_cast<H*>(static_cast<size_t>(kb));
            lds_add(bin, it - i1);
            lds_add(bin + 1, i1);
          }
        }
      }
    }
  }
  __syncthreads();

  // histogram rows out, row (sensor, forward tile) at ((s * n_atiles) + at) * wpa:
  // wave w takes rows w, w + 4, ..., 64 samples of a row per step, with the
  // LDS reads of eight rows (and their scales) issued before their
  // conversions and stores.  Row indices and addresses are wave-uniform;
  // each row is stored through a buffer resource over it, which drops the
  // lanes past its end.
  {
    constexpr int RB = 8;
    const int nrw = (min(NS, P.S - chunk * NS) - wave + 3) >> 2;   // this wave's rows
    for (int i0 = 0; i0 < P.wpa; i0 += 64) {
      const int i = i0 + lane;
      const int ic = i < P.wpa ? i : 0;   // (an in-row bin for the LDS read of lanes past the end)
      for (int r0 = 0; r0 < nrw; r0 += RB) {
        H hv[RB];
        double inv[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int jr = wave + 4 * (r0 + u < nrw ? r0 + u : 0);
          hv[u] = hist[jr * P.wpa + ic];
          inv[u] = inv_a[jr];
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int j = wave + 4 * (r0 + u);
          if (r0 + u < nrw)   // wave-uniform
            row_store(rows + ((size_t)(chunk * NS + j) * P.n_atiles + at) * P.wpa, P.wpa, i,
                      (T)((double)hv[u] * inv[u]));
        }
      }
    }
  }
  if (wave == 0 && s_ok) klo_tab[(size_t)s * P.n_atiles + at] = klo_a[lane];
}

// A through partial rows, pass 2: one work-group per (sensor, segment of kseg <= 256 samples),
// one sample per lane.  Each wave loads the window starts of the sensor's
// forward tiles, 256 at a time, picks by ballot the tiles whose row window
// overlaps its own 64 samples, and every lane adds its sample of those rows,
// in increasing tile order, in FP64 (kGatherLoads loads in flight, taken
// across the 256 tiles); then the work-group scales, writes y and forms
// the FP64 partial of ||y||^2.  No atomics: the result is the same on every
// run.  Rows and window starts are sensor-major, so one sensor's rows are
// contiguous.  The launch remaps work-groups so each XCD takes a contiguous
// run of sensors: at the 512x512 workload (four chunks of 64 sensors) those
// are rows pass 1 wrote on the same pair of XCDs, half of them in this
// XCD's own L2.
constexpr int kGatherLoads = 8;

__device__ __forceinline__ void gather_body(const OpParams& P, int blk, int pidx, const float* __restrict__ rows,
                                            const int* __restrict__ klo_tab, float* __restrict__ y,
                                            double* __restrict__ part_q) {
  using T = float;
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int s = __builtin_amdgcn_readfirstlane(blk / P.nseg);   // (uniform: keeps the row addresses scalar)
  const int seg = blk - s * P.nseg;
  const int k0 = seg * P.kseg;
  const int kn = min(P.kseg, P.K - k0);
  const int k = k0 + tid;
  const bool k_ok = tid < kn;
  const int* kt = klo_tab + (size_t)s * P.n_atiles;
  const T* srow = rows + (size_t)s * P.n_atiles * P.wpa;
  const int wlo = k0 + wave * 64, whi = min(k0 + kn, wlo + 64);  // this wave's samples
  double acc = 0.0;
  if (wlo < whi) {
    // Tiles go in groups of 256: the window starts of a group are loaded
    // together (four per lane, tile g0 + 64 c + lane), the four ballots pick
    // the tiles whose row overlaps this wave's samples, and the rows are read
    // kGatherLoads at a time across the group, in increasing tile order.
    for (int g0 = 0; g0 < P.n_atiles; g0 += 256) {
      int kl[4];
      uint64_t m[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int t = g0 + 64 * c + lane;
        kl[c] = t < P.n_atiles ? kt[t] : 0;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int t = g0 + 64 * c + lane;
        m[c] = __ballot(t < P.n_atiles && kl[c] < whi && kl[c] + P.wpa > wlo);
      }
      // m[0] and kl[0] belong to chunk c, the chunk of the next pick
      // (wave-uniform); advance() moves on to the next chunk with picks
      int c = 0;
      auto advance = [&]() {
        while (c < 4 && m[0] == 0) {
          m[0] = m[1];
          m[1] = m[2];
          m[2] = m[3];
          m[3] = 0;
          kl[0] = kl[1];
          kl[1] = kl[2];
          kl[2] = kl[3];
          ++c;
        }
      };
      advance();
      while (c < 4) {
        // every lane loads its sample of the row through a buffer resource
        // over the row, which reads zero for samples outside it, so the
        // loads go out back to back with no test (lanes past the segment's
        // end read what they read; their sums are never written)
        float v[kGatherLoads];
#pragma unroll
        for (int u = 0; u < kGatherLoads; ++u) {
          v[u] = 0.f;
          if (c < 4) {   // wave-uniform
            const int b = __builtin_ctzll(m[0]);
            m[0] &= m[0] - 1;
            const int klb = __builtin_amdgcn_readlane(kl[0], b);
            v[u] = trace_load(srow + (size_t)(g0 + 64 * c + b) * P.wpa, P.wpa, k - klb);
            advance();
          }
        }
#pragma unroll
        for (int u = 0; u < kGatherLoads; ++u) acc += (double)v[u];
      }
    }
  }
  const double scale = 2.0 * P.out_scale;   // (the rows hold sums of w x / 2)
  double q = 0.0;
  if (k_ok) {
    const T out = (T)(acc * scale);
    y[(size_t)s * P.K + k] = out;
    q = (double)out * (double)out;
  }
  if (part_q) {
    q = block_sum(q, red);
    if (tid == 0) part_q[pidx] = q;
  }
}

}  // namespace

}  // namespace pa
