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
constexpr int kSensorsPerFwdBlock = 64;  // forward operator: one sensor per lane of a wave
constexpr size_t kLdsPreferred = 64 * 1024 - 256;  // dynamic LDS that keeps several work-groups per CU
constexpr size_t kLdsMax = 160 * 1024 - 1024;      // gfx950: 160 KiB of LDS per work-group, minus static use
constexpr size_t kLdsPreferredFwd = 80 * 1024;      // forward pass 1: two work-groups per CU

// Everything a kernel needs about the operator, by value.  Lengths are in
// "sample units": metres multiplied by 1 / (c dt), so a distance equals its
// delay in samples.
struct OpParams {
  int32_t nx, ny, nz;       // image size
  int32_t S, K;             // sensors, samples
  double org[3];            // position of pixel (0,0,0), sample units
  double hs;                // pixel pitch, sample units
  double rmin;              // distance clamp, sample units
  double inv_cdt;           // metres -> sample units
  int32_t t0i;              // floor(t0 / dt)
  float t0f;                // t0 / dt - t0i, in [0, 1)
  double t0fd;
  const double* sensors;    // device, [S][ndim], metres
  int32_t ntile[3];         // base tiles per axis
  int32_t n_tiles;          // product
  int32_t wp;               // adjoint: LDS window stride (samples) of one sensor
  int32_t sc;               // adjoint: sensors staged per chunk
  int32_t msub[3];          // forward: base tiles per forward tile, per axis
  int32_t nsub;             // product
  int32_t natile[3];        // forward tiles per axis
  int32_t n_atiles;
  int32_t n_chunks;         // forward: sensor chunks of 64
  int32_t wpa;              // forward: LDS histogram stride of one sensor
  int32_t kseg;             // forward gather: samples per work-group (<= 256, one per lane)
  int32_t nseg;             // forward gather: segments per trace
  double near_r2;           // squared tile-centre distance (sample units) below which a
                            // sensor takes the FP64 delay path in the FP32 kernels
  float out_scale;          // converts accumulated kernel units to 1/metres (float path)
  double out_scale_d;       // same, double path
};

// LDS layouts, shared by the planner (sizes) and the kernels (offsets).
struct BpLayout {
  size_t sct, klo, sid, nd, win, total;
};
// sc sensors per chunk, wp samples per window row, elem bytes per sample;
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

struct FpLayout {
  size_t hist, pixtab, xs, klo, inv, total;
};
// Histogram bins have the element size elem: 32-bit fixed point for FP32,
// double for FP64.  inv: per-sensor inverse fixed-point scale and the
// per-base-tile sums of |x| that set it (FP32).
PA_HD inline FpLayout fp_layout(int wpa, int nsub, size_t elem, size_t pix_bytes) {
  FpLayout L;
  L.hist = 0;
  L.pixtab = align16((size_t)kSensorsPerFwdBlock * wpa * elem);
  L.xs = L.pixtab + (size_t)kBlock * pix_bytes;
  L.klo = L.xs + align16((size_t)nsub * kBlock * elem);
  L.inv = L.klo + align16(kSensorsPerFwdBlock * 4);
  // inv: per-sensor inverse scale, then the per-base-tile |x| partials of four waves
  L.total = L.inv + (kSensorsPerFwdBlock + 4 * (size_t)nsub) * sizeof(double);
  return L;
}

// forward gather: no dynamic LDS (each wave keeps its tile selection in registers)
PA_HD inline size_t gather_lds() { return 0; }

struct Plan {
  OpParams op;
  int ndim;
  pa_dtype dtype;
  size_t elem;              // sizeof(T)
  int64_t P, M;             // pixels, samples (S*K)
  size_t bp_lds, fp_lds, gather_lds;  // dynamic LDS bytes
  int bp_grid, fp_grid, gather_grid;
  size_t fwd_scratch;       // bytes of forward-operator scratch (partial rows + window table)
  size_t part_rows_off, klo_tab_off;  // offsets inside that scratch
};

// Tiling choices an autotuning run can fix for a geometry shape.  Zero
// fields leave the planner's own choice.
struct Tuning {
  int32_t fwd_tile[3];   // forward operator: base tiles per forward tile, per axis
  int32_t adj_lds;       // adjoint: LDS budget per work-group (bytes) that sets the sensor chunk
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
// Candidate tilings the autotuner times for a geometry of this ndim.
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
  int64_t scr;         // byte offset of the frame's forward partial rows in the scratch area
  int64_t scr_tab;     // byte offset of the frame's window-start table in the scratch area
  int32_t b_bp, n_bp;  // adjoint blocks (n_bp = 0 without pixels)
  int32_t b_fp, n_fp;  // forward pass-1 blocks (0 when the frame is empty)
  int32_t b_ga, n_ga;  // forward gather blocks (S * nseg whenever S * K > 0)
  int32_t b_m, n_m;    // BLAS blocks over the frame's S*K samples (>= 1)
  int32_t b_p, n_p;    // BLAS blocks over the frame's pixels (>= 1)
  int32_t s_bp;        // first slot of the frame's adjoint partials (max(n_bp, 1) slots)
  int32_t s_ga;        // first slot of the frame's gather partials (max(n_ga, 1) slots)
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
  std::vector<Plan> plans;        // caller order
  std::vector<FrameDesc> table;   // work order (largest first)
  std::vector<int64_t> xoff, yoff;  // caller order, nf + 1 prefix offsets (elements)
  int bp_grid = 0, fp_grid = 0, gather_grid = 0, m_grid = 0, p_grid = 0;
  int bp_slots = 0, ga_slots = 0;
  size_t bp_lds = 0, fp_lds = 0, gather_lds = 0;
  size_t fwd_scratch = 0;
  int64_t P_total = 0, M_total = 0;
  bool tuned = false;             // planned with the recorded per-frame tunings
};

// use_tuning: plan frames with their recorded tunings (capped so the batch's
// LDS stays within its rule plans' maximum) instead of by rule.
pa_status make_batch_plan(const pa_geometry* frames, int32_t n_frames, pa_dtype dtype, BatchPlan* bp,
                          std::string* msg, bool use_tuning = false);

// Workspace of batched calls: the device frame table, the forward scratch
// and (cg) the per-frame CGLS state for `iters` iterations, partials and vectors.
struct BatchLayout {
  size_t table, status, gamma, alpha, part_q, part_r, part_s, part_x, part_p, vec_r, vec_q, vec_s, vec_p, fwd, total;
  int astride;   // doubles per frame in gamma and alpha (iters + 2)
};
BatchLayout batch_layout(const BatchPlan& bp, int32_t iters, bool cg);

// Sizes of the BLAS-1 grids (fixed per vector length so every reduction runs
// in the same order every time).
int blas_grid(int64_t n);

// CGLS workspace layout.
struct CglsLayout {
  size_t status, gamma, alpha, part_q, part_r, part_s, part_x, part_p, vec_r, vec_q, vec_s, vec_p, fwd, total;
  int g_q, g_m, g_p, g_bp;  // partial counts: forward gather, over S*K, over pixels, adjoint tiles
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
