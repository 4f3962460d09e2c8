// Host-side planning shared by every entry point: validation of a geometry,
// conversion to sample units, tiling and LDS budgets.  Plain C++ with no HIP
// calls, so it runs (and is tested) without a GPU.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "pa.h"

#ifdef __HIPCC__
#define PA_HD __host__ __device__
#else
#define PA_HD
#endif

namespace pa {

PA_HD inline size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

// Base tiles: one work-group of 256 lanes, one pixel per lane.
//   2D: 16 x 16 x 1      3D: 8 x 8 x 4
template <int ND> struct Tile;
template <> struct Tile<2> { static constexpr int X = 16, Y = 16, Z = 1; };
template <> struct Tile<3> { static constexpr int X = 8, Y = 8, Z = 4; };

constexpr int kBlock = 256;          // lanes per work-group, every kernel
constexpr size_t kLdsPreferred = 64 * 1024 - 256;  // dynamic LDS that keeps several work-groups per CU
constexpr size_t kLdsMax = 160 * 1024 - 1024;      // gfx950: 160 KiB of LDS per work-group, minus static use
constexpr int kFwdList = kBlock;     // forward operator: base tiles listed per round (one per lane)
constexpr int kSensorsPerFwdBlock = 64;          // partial-row forward: one sensor per lane of a wave
constexpr size_t kLdsPreferredFwd = 80 * 1024;   // partial-row forward pass 1: two work-groups per CU
constexpr size_t kLdsBatchFwd = 46 * 1024;       // batched sensor-major forward: with its 1 KiB of static
                                                  // LDS within 48 KiB, three work-groups per CU

// Arithmetic of a dtype: the type of every vector element (images, traces,
// CGLS vectors) and of the per-pair delay and weight.
PA_HD inline bool data_is_f32(pa_dtype d) { return d == PA_F32; }
PA_HD inline bool phase_is_f32(pa_dtype d) { return d != PA_F64; }

// Everything a kernel needs about the operator, by value.  Lengths are in
// "sample units": metres multiplied by 1 / (c dt), so a distance equals its
// delay in samples.
struct OpParams {
  int32_t nx, ny, nz;       // image size
  int32_t S, K;             // sensors, samples
  double org[3];            // position of pixel (0,0,0), sample units
  double hs;                // pixel pitch, sample units
  float hs2h;               // hs^2 / 2 in FP32 (the FP32 phase's |o|^2 / 2 = (hs^2 / 2) |u|^2 term)
  double rmin;              // distance clamp, sample units
  double inv_cdt;           // metres -> sample units
  int32_t t0i;              // floor(t0 / dt)
  float t0f;                // t0 / dt - t0i, in [0, 1)
  double t0fd;
  const double* sensors;    // device, [S][ndim], metres
  int32_t ntile[3];         // base tiles per axis
  int32_t n_tiles;          // product
  int32_t wp;               // samples of one sensor's window over a base tile: every tap of every
                            // pixel of the tile lies in [klo, klo + wp) (adjoint: LDS row stride)
  int32_t sc;               // adjoint: sensors staged per chunk
  int32_t fseg;             // forward: samples of one trace owned by a work-group
  int32_t fnseg;            // forward: segments per trace (work-groups per sensor)
  int32_t fbins;            // forward: histogram bins per wave, fseg + 2 wp + 2
  int32_t ffix;             // forward, FP32 delay arithmetic: 1 = fixed-point tile rows, 0 = FP64 bins
  // forward through partial rows (PA_F32 with a workspace): pass 1 scatters
  // one forward tile for 64 sensors into LDS rows, pass 2 adds the rows up
  int32_t msub[3];          // base tiles per forward tile, per axis
  int32_t nsub;             // product
  int32_t natile[3];        // forward tiles per axis
  int32_t n_atiles;
  int32_t n_chunks;         // sensor chunks of 64
  int32_t wpa;              // LDS row stride of one sensor over a forward tile
  int32_t kseg;             // pass 2: samples per work-group (<= 256, one per lane)
  int32_t nseg;             // pass 2: segments per trace
  double near_r2;           // squared tile-centre distance (sample units) below which a
                            // sensor takes the FP64 delay path in the FP32-phase kernels
  double out_scale;         // converts sums of tap weights w = 1 / R to 1/metres
};

// LDS layouts, shared by the planner (sizes) and the kernels (offsets).
struct BpLayout {
  size_t sct, klo, sid, nd, win, total;
};
// sc sensors per chunk, wp entries per window row, elem bytes per entry (a
// sample and its difference to the next);
// sc_bytes per-sensor constants; near_bytes per-sensor FP64 table (0 in FP64 kernels).
PA_HD inline BpLayout bp_layout(int sc, int wp, size_t elem, size_t sc_bytes, size_t near_bytes) {
  BpLayout L;
  L.sct = 0;
  L.klo = align16((size_t)sc * sc_bytes);
  L.sid = L.klo + align16((size_t)sc * 4);
  L.nd = L.sid + align16((size_t)sc * 4);
  L.win = L.nd + align16((size_t)sc * near_bytes);
  L.total = L.win + (size_t)sc * wp * elem;
  return L;
}

// Sensor-major forward operator, per listed base tile: the offset of its
// window in the segment's histogram, near flag and the factor that turns the
// tile's sum of |x| into a bound on any partial sum of its taps.
struct FpTile {
  int32_t off;     // first bin of the tile's window in the FP64 histogram
  int32_t xoff;    // index in x of the tile's first pixel
  int32_t lim;     // pixels of the tile inside the image per axis: nx | ny << 8 | nz << 16,
                   // plus kFpNear when the sensor takes the FP64 delay path (FP32-phase kernels)
  float ib;        // 1 / (2 max(dmin, r_min)), dmin = distance from the sensor to the tile's box
};
constexpr int32_t kFpNear = 1 << 24;

// The forward operator's per-(tile, sensor) delay constants with FP32 delay
// arithmetic: the far-pair fields of the adjoint's constants (the same values
// for the same tile and sensor).
struct FpSC32 {
  float E, DXH, DYH, DZH, KRN, KR2;
  int32_t BASE;
  int32_t pad;
};

constexpr int kFwdGroupMax = 8;  // forward: list entries a wave processes together (one fixed-point scale):
                                 // 8 with float vectors, 4 with double

// Forward operator LDS: a list of up to kFwdList base tiles with their
// per-(tile, sensor) constants (sc_bytes each), one FP64 histogram of fbins
// bins per wave and, with fixed-point rows (fix), one int row of fbins bins
// per wave.
struct FpLayout {
  size_t lst, ltab, hist, irow, total;
};
PA_HD inline FpLayout fp_layout(int fbins, int wp, size_t sc_bytes, bool fix) {
  (void)wp;
  FpLayout L;
  L.lst = 0;
  L.ltab = align16((size_t)kFwdList * sc_bytes);
  L.hist = L.ltab + align16((size_t)kFwdList * sizeof(FpTile));
  L.irow = L.hist + 4 * (size_t)fbins * sizeof(double);
  L.total = L.irow + (fix ? 4 * align16((size_t)fbins * 4) : 0);
  return L;
}

// Partial-row forward operator, pass 1 LDS: 32-bit fixed-point rows of 64
// sensors, the pixel offsets of a base tile, the forward tile's x values, the
// rows' window starts and the per-sensor scales.
struct Fp2Layout {
  size_t hist, xs, klo, inv, total;
};
PA_HD inline Fp2Layout fp2_layout(int wpa, int nsub) {
  Fp2Layout L;
  L.hist = 0;
  // xs has four entries of slack: the scatter loop reads four pixels ahead
  // without a bounds test
  L.xs = align16((size_t)kSensorsPerFwdBlock * wpa * 4);
  L.klo = L.xs + align16(((size_t)nsub * kBlock + 4) * 4);
  L.inv = L.klo + align16(kSensorsPerFwdBlock * 4);
  // inv: row scales [64], per-wave sums of |x| [nsub][4], bound terms
  // [nsub][64] (doubles), then the fixed-point scales [64] (floats)
  L.total = L.inv + (kSensorsPerFwdBlock + 4 * (size_t)nsub + (size_t)nsub * kSensorsPerFwdBlock) * sizeof(double) +
            kSensorsPerFwdBlock * sizeof(float);
  return L;
}

struct Plan {
  OpParams op;
  int ndim;
  pa_dtype dtype;
  size_t elem;              // bytes of one vector element
  int64_t P, M;             // pixels, samples (S*K)
  size_t bp_lds, fp_lds;    // dynamic LDS bytes
  int bp_grid, fp_grid;     // adjoint: one work-group per base tile; forward: one per (sensor, segment)
  // partial-row forward (PA_F32): used where a workspace is given and two_pass is set
  bool two_pass;
  size_t fp2_lds;
  int fp2_grid, gather_grid;
  size_t fwd_scratch;       // workspace bytes for the partial rows and their window starts (0: not used)
  size_t part_rows_off, klo_tab_off;
};

// Tiling choices an autotuning run can fix for a geometry shape.  Zero
// fields leave the planner's own choice.
struct Tuning {
  int32_t fwd_seg;       // forward operator: samples of a trace per work-group
  int32_t adj_lds;       // adjoint: LDS budget per work-group (bytes) that sets the sensor chunk
  int32_t fwd_mode;      // forward, FP32 delay arithmetic: 1 = fixed-point tile rows, 2 = FP64 bins,
                         // 3 = partial rows (PA_F32 with a workspace)
  int32_t fwd_tile[3];   // partial-row forward: base tiles per forward tile, per axis
};

// Fills *plan from g.  Returns PA_OK or an error with *msg set.  Never touches
// the GPU or dereferences g->sensors.  With force == nullptr the planner uses
// the tuning recorded for g's shape (see tune_store), if any.
pa_status make_plan(const pa_geometry* g, pa_dtype dtype, Plan* plan, std::string* msg,
                    const Tuning* force = nullptr);

// Process-wide table of tunings keyed by shape (ndim, dtype, sizes, S, K and
// the pixel pitch in samples); thread-safe.
void tune_store(const pa_geometry* g, pa_dtype dtype, const Tuning& t);
bool tune_lookup(const pa_geometry* g, pa_dtype dtype, Tuning* t);
void tune_clear();
// Changes whenever the table does: anything cached from a plan (captured
// graphs) is stale once the epoch it was made under has passed.
uint64_t tune_epoch();
// Candidate tilings the autotuner times.
int fwd_seg_candidates(int32_t* out, int max);
int fwd_tile_candidates(int ndim, int (*out)[3], int max);
int adj_lds_candidates(size_t* out, int max);

// One frame of a batch as the batched kernels see it (device table, sorted
// by work, largest first).  Block ranges [b_*, b_* + n_*) are those of each
// batched launch; partial sums go to the frame's own slot range, at the same
// local index as in a single-frame call, so every frame's sums are formed in
// the same order as when it is solved alone.
struct FrameDesc {
  OpParams op;
  int64_t xo, yo;      // element offsets of the frame's image / traces in the packed buffers
  int32_t b_bp, n_bp;  // adjoint blocks (n_bp = 0 without pixels)
  int32_t b_fp, n_fp;  // forward blocks (S * fnseg whenever S * K > 0, pixels or not)
  int32_t b_m, n_m;    // BLAS blocks over the frame's S*K samples (>= 1)
  int32_t b_p, n_p;    // BLAS blocks over the frame's pixels (>= 1)
  int32_t s_bp;        // first slot of the frame's adjoint partials (max(n_bp, 1) slots)
  int32_t s_fp;        // first slot of the frame's forward partials (max(n_fp, 1) slots)
  int32_t frame;       // position in the caller's frame order
  int32_t pad;
};

// Host plan of a batch: per-frame plans (caller order), the device table
// (work order) and the grid and buffer totals.
struct BatchPlan {
  int nf = 0;
  int ndim = 2;
  pa_dtype dtype = PA_F32;
  size_t elem = 4;
  bool frac = false;
  bool ffix = false;              // forward accumulation mode shared by every frame
  std::vector<Plan> plans;        // caller order
  std::vector<FrameDesc> table;   // work order (largest first)
  std::vector<int64_t> xoff, yoff;  // caller order, nf + 1 prefix offsets (elements)
  int bp_grid = 0, fp_grid = 0, m_grid = 0, p_grid = 0;
  int bp_slots = 0, fp_slots = 0;
  size_t bp_lds = 0, fp_lds = 0;
  int64_t P_total = 0, M_total = 0;
  bool tuned = false;             // planned with the recorded per-frame tunings
};

// use_tuning: plan frames with their recorded tunings (capped so the batch's
// LDS stays within its rule plans' maximum) instead of by rule.
pa_status make_batch_plan(const pa_geometry* frames, int32_t n_frames, pa_dtype dtype, BatchPlan* bp,
                          std::string* msg, bool use_tuning = false);

// Workspace of batched calls: the device frame table and (cg) the per-frame
// CGLS state for `iters` iterations, partials and vectors.
struct BatchLayout {
  size_t table, status, gamma, alpha, part_q, part_r, part_s, part_x, part_p, vec_r, vec_q, vec_s, vec_p, total;
  int astride;   // doubles per frame in gamma and alpha (iters + 2)
};
BatchLayout batch_layout(const BatchPlan& bp, int32_t iters, bool cg);

// Sizes of the BLAS-1 grids (fixed per vector length so every reduction runs
// in the same order every time).
int blas_grid(int64_t n);

// CGLS workspace layout.
struct CglsLayout {
  size_t status, gamma, alpha, part_q, part_r, part_s, part_x, part_p, vec_r, vec_q, vec_s, vec_p, vec_p2, fwd, total;
  int g_q, g_m, g_p, g_bp;  // partial counts: forward work-groups, over S*K, over pixels, adjoint tiles
  bool fused;               // the direction update rides on the partial-row forward (p alternates vec_p, vec_p2)
  int g_pf;                 // ... and ||p||^2 then has one partial per forward tile
};
CglsLayout cgls_layout(const Plan& plan, int32_t iters);

// Landweber workspace layout.
struct LwLayout {
  size_t status, alpha0, sigma2, omega, part_r, part_s, part_x, part_n, vec_r, vec_q, vec_s, vec_v, fwd, total;
  int g_m, g_p, g_bp;
};
LwLayout lw_layout(const Plan& plan);

// Proximal-gradient (FISTA) workspace layout: the Landweber fields (status,
// step and eigenvalue at the same offsets) plus the TV and l1 partials and
// the two extrapolated points z_k, z_{k+1} used alternately.
struct FistaLayout {
  LwLayout lw;
  size_t part_tv, part_l1, vec_z0, vec_z1, total;
};
FistaLayout fista_layout(const Plan& plan);

}  // namespace pa
