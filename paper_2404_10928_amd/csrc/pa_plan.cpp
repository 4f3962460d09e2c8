// Host-side validation, unit conversion and tiling (no GPU access).
#include "pa_plan.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>

namespace pa {

namespace {

bool finite(double v) { return std::isfinite(v); }

pa_status fail(std::string* msg, pa_status st, const char* text) {
  if (msg) *msg = text;
  return st;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace

int blas_grid(int64_t n) {
  int64_t g = (n + 1023) / 1024;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1024));
}

namespace {

struct TuneKey {
  int32_t ndim, dtype, nx, ny, nz, S, K;
  uint64_t hs_bits;
  bool operator<(const TuneKey& o) const {
    return std::tie(ndim, dtype, nx, ny, nz, S, K, hs_bits) < std::tie(o.ndim, o.dtype, o.nx, o.ny, o.nz, o.S, o.K, o.hs_bits);
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, Tuning>* g_tune = nullptr;
uint64_t g_tune_epoch = 0;   // bumped whenever the table changes

TuneKey tune_key(const pa_geometry* g, pa_dtype dtype) {
  TuneKey k{g->ndim, (int32_t)dtype, g->nx, g->ny, g->nz, g->n_sensors, g->n_samples, 0};
  const double hs = g->h / (g->c * g->dt);
  std::memcpy(&k.hs_bits, &hs, sizeof(hs));
  return k;
}

}  // namespace

void tune_store(const pa_geometry* g, pa_dtype dtype, const Tuning& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune) g_tune = new std::map<TuneKey, Tuning>();
  (*g_tune)[tune_key(g, dtype)] = t;
  ++g_tune_epoch;
}

bool tune_lookup(const pa_geometry* g, pa_dtype dtype, Tuning* t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune) return false;
  auto it = g_tune->find(tune_key(g, dtype));
  if (it == g_tune->end()) return false;
  *t = it->second;
  return true;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune) g_tune->clear();
  ++g_tune_epoch;
}

uint64_t tune_epoch() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tune_epoch;
}

int fwd_seg_candidates(int32_t* out, int max) {
  static const int32_t c[] = {128, 256, 384, 512, 640, 768, 1024};
  const int n = std::min(7, max);
  for (int i = 0; i < n; ++i) out[i] = c[i];
  return n;
}

int fwd_tile_candidates(int ndim, int (*out)[3], int max) {
  static const int c2[][3] = {{1, 1, 1}, {2, 1, 1}, {2, 2, 1}, {4, 2, 1}};
  static const int c3[][3] = {{1, 1, 1}, {2, 1, 2}, {2, 2, 2}, {2, 2, 4}};
  const int (*c)[3] = ndim == 2 ? c2 : c3;
  const int n = std::min(4, max);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) out[i][a] = c[i][a];
  return n;
}

int adj_lds_candidates(size_t* out, int max) {
  static const size_t c[] = {24 * 1024, 40 * 1024, kLdsPreferred, 96 * 1024};
  const int n = std::min(4, max);
  for (int i = 0; i < n; ++i) out[i] = c[i];
  return n;
}

pa_status make_plan(const pa_geometry* g, pa_dtype dtype, Plan* plan, std::string* msg, const Tuning* force) {
  if (!g) return fail(msg, PA_ERR_INVALID_ARGUMENT, "geometry pointer is NULL");
  if (!plan) return fail(msg, PA_ERR_INVALID_ARGUMENT, "plan pointer is NULL");
  if (dtype != PA_F32 && dtype != PA_F64 && dtype != PA_MIXED)
    return fail(msg, PA_ERR_INVALID_ARGUMENT, "dtype must be PA_F32, PA_F64 or PA_MIXED");
  if (g->ndim != 2 && g->ndim != 3) return fail(msg, PA_ERR_INVALID_ARGUMENT, "ndim must be 2 or 3");
  if (g->nx < 0 || g->ny < 0 || g->nz < 0) return fail(msg, PA_ERR_INVALID_ARGUMENT, "image sizes must be >= 0");
  if (g->ndim == 2 && g->nz != 1) return fail(msg, PA_ERR_INVALID_ARGUMENT, "nz must be 1 for a 2D geometry");
  if (g->n_sensors < 0 || g->n_samples < 0) return fail(msg, PA_ERR_INVALID_ARGUMENT, "n_sensors and n_samples must be >= 0");
  if (!finite(g->h) || !(g->h > 0)) return fail(msg, PA_ERR_INVALID_ARGUMENT, "h must be finite and > 0");
  if (!finite(g->dt) || !(g->dt > 0)) return fail(msg, PA_ERR_INVALID_ARGUMENT, "dt must be finite and > 0");
  if (!finite(g->c) || !(g->c > 0)) return fail(msg, PA_ERR_INVALID_ARGUMENT, "c must be finite and > 0");
  if (!finite(g->t0)) return fail(msg, PA_ERR_INVALID_ARGUMENT, "t0 must be finite");
  if (!finite(g->r_min) || g->r_min < 0) return fail(msg, PA_ERR_INVALID_ARGUMENT, "r_min must be finite and >= 0");
  for (int a = 0; a < 3; ++a)
    if (!finite(g->center[a])) return fail(msg, PA_ERR_INVALID_ARGUMENT, "center must be finite");
  if (g->n_sensors > 0 && !g->sensors) return fail(msg, PA_ERR_INVALID_ARGUMENT, "sensors is NULL but n_sensors > 0");
  if (g->sensors && (reinterpret_cast<uintptr_t>(g->sensors) % 8) != 0)
    return fail(msg, PA_ERR_INVALID_ARGUMENT, "sensors must be 8-byte aligned");

  Tuning tuned{0, 0, 0, {0, 0, 0}};
  if (force) tuned = *force;
  else (void)tune_lookup(g, dtype, &tuned);

  const int64_t P = (int64_t)g->nx * g->ny * g->nz;
  const int64_t M = (int64_t)g->n_sensors * g->n_samples;
  if (P > std::numeric_limits<int32_t>::max()) return fail(msg, PA_ERR_UNSUPPORTED, "more than 2^31-1 pixels");
  if (M > std::numeric_limits<int32_t>::max()) return fail(msg, PA_ERR_UNSUPPORTED, "n_sensors * n_samples exceeds 2^31-1");
  if (g->n_samples > (1 << 22)) return fail(msg, PA_ERR_UNSUPPORTED, "n_samples above 2^22");

  const double inv_cdt = 1.0 / (g->c * g->dt);
  const double hs = g->h * inv_cdt;
  const double T0 = g->t0 / g->dt;
  if (!finite(inv_cdt) || !finite(hs) || !(hs > 0)) return fail(msg, PA_ERR_INVALID_ARGUMENT, "h / (c dt) is not a finite positive number");
  if (std::fabs(T0) > (double)(1 << 30)) return fail(msg, PA_ERR_UNSUPPORTED, "|t0 / dt| above 2^30");

  Plan& pl = *plan;
  pl = Plan{};
  pl.ndim = g->ndim;
  pl.dtype = dtype;
  pl.elem = data_is_f32(dtype) ? 4 : 8;
  pl.P = P;
  pl.M = M;
  OpParams& op = pl.op;
  op.nx = g->nx;
  op.ny = g->ny;
  op.nz = g->nz;
  op.S = g->n_sensors;
  op.K = g->n_samples;
  op.hs = hs;
  op.hs2h = (float)(0.5 * hs * hs);
  op.inv_cdt = inv_cdt;
  op.rmin = (g->r_min > 0 ? g->r_min : 0.5 * g->h) * inv_cdt;
  const double t0i = std::floor(T0);
  op.t0i = (int32_t)t0i;
  op.t0fd = T0 - t0i;
  op.t0f = (float)op.t0fd;
  if (op.t0f >= 1.0f) {  // rounding pushed the fraction to 1: carry it
    op.t0i += 1;
    op.t0fd = 0.0;
    op.t0f = 0.0f;
  }
  op.sensors = g->sensors;
  const int nd = g->ndim;
  for (int a = 0; a < 3; ++a) {
    int n = a == 0 ? g->nx : a == 1 ? g->ny : g->nz;
    double c = (a < nd) ? g->center[a] : 0.0;
    op.org[a] = (c - 0.5 * (n - 1) * g->h) * inv_cdt;
  }
  if (nd == 2) op.org[2] = 0.0;

  const int TX = nd == 2 ? Tile<2>::X : Tile<3>::X;
  const int TY = nd == 2 ? Tile<2>::Y : Tile<3>::Y;
  const int TZ = nd == 2 ? Tile<2>::Z : Tile<3>::Z;
  op.ntile[0] = ceil_div(g->nx, TX);
  op.ntile[1] = ceil_div(g->ny, TY);
  op.ntile[2] = ceil_div(g->nz, TZ);
  op.n_tiles = op.ntile[0] * op.ntile[1] * op.ntile[2];

  const size_t elem = pl.elem;
  const bool p32 = phase_is_f32(dtype);
  const size_t sc_bytes = p32 ? 48 : 64;     // per-(tile, sensor) constants in LDS (adjoint)
  const size_t fsc_bytes = p32 ? sizeof(FpSC32) : 64;  // the same for the forward operator's list
  const size_t near_bytes = p32 ? 32 : 0;    // FP64 sensor vector + reference (FP32 near path)

  // Sensors closer than three base-tile half-diagonals to a tile centre take
  // the FP64 delay path in the FP32 kernels (the tile-local FP32 form loses
  // relative precision in R^2 when R is small against the tile size).  The
  // radius also covers r_min + a half-diagonal, so every pixel of a far pair
  // is more than r_min from its sensor and the FP32 path needs no clamp.
  {
    double ex = (TX - 1) * hs, ey = (TY - 1) * hs, ez = (TZ - 1) * hs;
    double hd = 0.5 * std::sqrt(ex * ex + ey * ey + ez * ez);
    double nr = std::max(3.0 * hd + 2.0, op.rmin + hd + 1.0);
    op.near_r2 = nr * nr;
  }

  // Adjoint: window of one sensor over the base tile's pixel-centre box.  Any
  // two pixels of the box differ in distance by at most its diagonal; the
  // margins cover floor(), the second tap and FP32 rounding of the delay.
  {
    double ex = (TX - 1) * hs, ey = (TY - 1) * hs, ez = (TZ - 1) * hs;
    double diag = std::sqrt(ex * ex + ey * ey + ez * ez);
    if (diag > 1e6) return fail(msg, PA_ERR_UNSUPPORTED, "pixel pitch spans too many samples");
    op.wp = (int32_t)std::ceil(diag) + 5;
    const size_t per = sc_bytes + 8 + near_bytes + (size_t)op.wp * 2 * elem;   // window entries: sample pairs
    const size_t slack = 64;  // alignment of the four LDS arrays
    const size_t budget = tuned.adj_lds > 0 ? std::min<size_t>((size_t)tuned.adj_lds, kLdsMax) : 40 * 1024;
    int64_t sc_max = budget > slack ? (int64_t)((budget - slack) / per) : 0;
    if (sc_max < 1) sc_max = (int64_t)((kLdsPreferred - slack) / per);
    if (sc_max < 1) sc_max = (int64_t)((kLdsMax - slack) / per);
    if (sc_max < 1) return fail(msg, PA_ERR_UNSUPPORTED, "trace window of one tile does not fit in LDS (h / (c dt) too large)");
    sc_max = std::min<int64_t>(sc_max, kBlock);
    int64_t S = std::max<int64_t>(g->n_sensors, 1);
    int64_t nchunk = (S + sc_max - 1) / sc_max;
    op.sc = (int32_t)((S + nchunk - 1) / nchunk);
    pl.bp_lds = bp_layout(op.sc, op.wp, 2 * elem, sc_bytes, near_bytes).total;
    if (pl.bp_lds > kLdsMax) return fail(msg, PA_ERR_UNSUPPORTED, "adjoint LDS plan exceeds 160 KiB");
  }

  // Forward: one work-group per (sensor, segment of fseg samples).  It lists
  // the base tiles whose window reaches its segment and scatters their
  // pixels' taps into one FP64 histogram per wave covering the segment plus
  // a window's margin on either side.  The segment is the tuned one, else
  // the longest candidate that still gives at least 512 work-groups (two per
  // CU), and never more than the trace.
  {
    op.ffix = p32 && tuned.fwd_mode != 2 ? 1 : 0;
    const bool fix = op.ffix != 0;
    auto bins = [&](int32_t seg) { return seg + 2 * op.wp + 2; };
    auto fits = [&](int32_t seg) { return fp_layout(bins(seg), op.wp, fsc_bytes, fix).total <= kLdsMax; };
    const int64_t Kp = std::max<int64_t>(g->n_samples, 1);
    int32_t seg = 0;
    if (tuned.fwd_seg > 0 && fits(tuned.fwd_seg)) seg = tuned.fwd_seg;
    if (seg == 0) {
      int32_t cand[8];
      const int nc = fwd_seg_candidates(cand, 8);
      for (int i = nc - 1; i >= 0 && seg == 0; --i) {
        const int64_t wg = (int64_t)g->n_sensors * ((Kp + cand[i] - 1) / cand[i]);
        if ((wg >= 512 || i == 0) && fits(cand[i])) seg = cand[i];
      }
      for (int i = 0; i < nc && seg == 0; ++i)
        if (fits(cand[i])) seg = cand[i];
    }
    if (seg == 0) return fail(msg, PA_ERR_UNSUPPORTED, "forward histogram does not fit in LDS (h / (c dt) too large)");
    op.fseg = (int32_t)std::min<int64_t>(seg, Kp);
    op.fnseg = ceil_div(Kp, op.fseg);
    op.fbins = bins(op.fseg);
    pl.fp_lds = fp_layout(op.fbins, op.wp, fsc_bytes, fix).total;
  }

  // Partial-row forward (PA_F32 only, chosen by autotuning): the histogram
  // window of one sensor over a forward tile of msub base tiles; the tuned
  // forward tile if it fits, else the largest candidate whose LDS keeps two
  // work-groups per CU.  Unavailable (two_pass stays false) if none fits.
  if (dtype == PA_F32) {
    auto try_tile = [&](const int* m, size_t budget) {
      if (!(nd == 3 || m[2] == 1)) return false;
      double ex = (m[0] * TX - 1) * hs, ey = (m[1] * TY - 1) * hs, ez = (m[2] * TZ - 1) * hs;
      double diag = std::sqrt(ex * ex + ey * ey + ez * ez);
      if (diag > 1e6) return false;
      const int32_t wpa = ((int32_t)std::ceil(diag) + 5) | 1;  // odd stride spreads lanes over LDS banks
      const int nsub = m[0] * m[1] * m[2];
      const size_t lds = fp2_layout(wpa, nsub).total;
      if (lds > budget) return false;
      for (int a = 0; a < 3; ++a) op.msub[a] = m[a];
      op.nsub = nsub;
      op.wpa = wpa;
      pl.fp2_lds = lds;
      return true;
    };
    bool ok = tuned.fwd_tile[0] > 0 && tuned.fwd_tile[1] > 0 && tuned.fwd_tile[2] > 0 &&
              try_tile(tuned.fwd_tile, kLdsMax);
    int cand[4][3];
    const int nc = fwd_tile_candidates(nd, cand, 4);
    for (size_t budget : {kLdsPreferredFwd, kLdsMax})
      for (int ci = nc - 1; ci >= 0 && !ok; --ci) ok = try_tile(cand[ci], budget);
    if (ok) {
      for (int a = 0; a < 3; ++a) op.natile[a] = ceil_div(op.ntile[a], op.msub[a]);
      op.n_atiles = op.natile[0] * op.natile[1] * op.natile[2];
      op.n_chunks = ceil_div(g->n_sensors, kSensorsPerFwdBlock);
      op.kseg = std::max(1, std::min<int32_t>(g->n_samples, kBlock));
      op.nseg = g->n_samples > 0 ? ceil_div(g->n_samples, op.kseg) : 0;
      const size_t rows = (size_t)op.n_atiles * (size_t)g->n_sensors * (size_t)op.wpa * 4;
      const size_t tab = (size_t)op.n_atiles * (size_t)g->n_sensors * 4;
      pl.part_rows_off = 0;
      pl.klo_tab_off = align_up(rows, 256);
      const size_t scr = align_up(pl.klo_tab_off + tab, 256);
      const bool empty = P == 0 || M == 0;
      if (!empty && scr <= ((size_t)1 << 40)) {
        pl.fwd_scratch = scr;
        pl.fp2_grid = op.n_atiles * op.n_chunks;
        pl.gather_grid = g->n_sensors * op.nseg;
        pl.two_pass = tuned.fwd_mode == 3;
      }
    }
  }

  op.out_scale = inv_cdt;
  // The adjoint runs whenever there are pixels (with no sensors or samples it
  // writes zeros, and its CGLS epilogue still has work); the forward
  // operator whenever there are samples to write (with no pixels its
  // work-groups list no tile and write zeros).
  pl.bp_grid = P == 0 ? 0 : op.n_tiles;
  const int64_t fwg = M == 0 ? 0 : (int64_t)g->n_sensors * op.fnseg;
  if (fwg > std::numeric_limits<int32_t>::max()) return fail(msg, PA_ERR_UNSUPPORTED, "forward grid above 2^31-1 work-groups");
  pl.fp_grid = (int)fwg;
  return PA_OK;
}

CglsLayout cgls_layout(const Plan& plan, int32_t iters) {
  CglsLayout L{};
  const size_t A = 256;
  L.g_q = std::max(plan.two_pass ? plan.gather_grid : plan.fp_grid, 1);
  L.g_m = blas_grid(plan.M);
  L.g_p = blas_grid(plan.P);
  L.g_bp = std::max(plan.op.n_tiles, 1);
  L.fused = plan.dtype == PA_F32 && plan.two_pass && plan.fwd_scratch > 0 && plan.fp2_grid > 0 && plan.P > 0;
  L.g_pf = L.fused ? std::max(plan.op.n_atiles, 1) : 0;
  size_t off = 0;
  L.status = off; off = align_up(off + 64, A);
  L.gamma = off; off = align_up(off + sizeof(double) * (size_t)(iters + 2), A);
  L.alpha = off; off = align_up(off + sizeof(double) * (size_t)(iters + 2), A);
  L.part_q = off; off = align_up(off + sizeof(double) * L.g_q, A);
  L.part_r = off; off = align_up(off + sizeof(double) * L.g_m, A);
  L.part_s = off; off = align_up(off + sizeof(double) * L.g_bp, A);
  L.part_x = off; off = align_up(off + sizeof(double) * L.g_bp, A);
  L.part_p = off; off = align_up(off + sizeof(double) * std::max(L.g_p, L.g_pf), A);
  L.vec_r = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.M, 1), A);
  L.vec_q = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.M, 1), A);
  L.vec_s = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.P, 1), A);
  L.vec_p = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.P, 1), A);
  L.vec_p2 = off; off = align_up(off + (L.fused ? plan.elem * (size_t)plan.P : 0), A);
  L.fwd = off; off = align_up(off + (plan.two_pass ? plan.fwd_scratch : 0), A);
  L.total = off;
  return L;
}

LwLayout lw_layout(const Plan& plan) {
  LwLayout L{};
  const size_t A = 256;
  L.g_m = blas_grid(plan.M);
  L.g_p = blas_grid(plan.P);
  L.g_bp = std::max(plan.op.n_tiles, 1);
  size_t off = 0;
  L.status = off; off += 64;
  L.alpha0 = off; off += 8;
  L.sigma2 = off; off += 8;
  L.omega = off; off = align_up(off + 8, A);
  L.part_r = off; off = align_up(off + sizeof(double) * L.g_m, A);
  L.part_s = off; off = align_up(off + sizeof(double) * L.g_bp, A);
  L.part_x = off; off = align_up(off + sizeof(double) * L.g_bp, A);
  L.part_n = off; off = align_up(off + sizeof(double) * L.g_p, A);
  L.vec_r = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.M, 1), A);
  L.vec_q = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.M, 1), A);
  L.vec_s = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.P, 1), A);
  L.vec_v = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.P, 1), A);
  L.fwd = off; off = align_up(off + (plan.two_pass ? plan.fwd_scratch : 0), A);
  L.total = off;
  return L;
}

FistaLayout fista_layout(const Plan& plan) {
  FistaLayout F{};
  const size_t A = 256;
  F.lw = lw_layout(plan);
  size_t off = F.lw.total;
  F.part_tv = off; off = align_up(off + sizeof(double) * F.lw.g_p, A);
  F.part_l1 = off; off = align_up(off + sizeof(double) * F.lw.g_p, A);
  F.vec_z0 = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.P, 1), A);
  F.vec_z1 = off; off = align_up(off + plan.elem * (size_t)std::max<int64_t>(plan.P, 1), A);
  F.total = off;
  return F;
}

pa_status make_batch_plan(const pa_geometry* frames, int32_t n_frames, pa_dtype dtype, BatchPlan* bp,
                          std::string* msg, bool use_tuning) {
  if (!bp) return fail(msg, PA_ERR_INVALID_ARGUMENT, "batch plan pointer is NULL");
  if (n_frames < 1) return fail(msg, PA_ERR_INVALID_ARGUMENT, "a batch needs at least one frame");
  if (!frames) return fail(msg, PA_ERR_INVALID_ARGUMENT, "frame array is NULL");
  if (n_frames > (1 << 16)) return fail(msg, PA_ERR_UNSUPPORTED, "more than 65536 frames");
  BatchPlan B;
  B.nf = n_frames;
  B.dtype = dtype;
  B.plans.resize(n_frames);
  // A batched launch gives every work-group the largest LDS any frame needs,
  // so with use_tuning a frame keeps its tuned tiling only if that stays
  // within what the planner's rules give for the batch.
  // The rule plans of a batch also keep the forward's LDS within
  // kLdsBatchFwd (three work-groups per CU): a batched launch mixes frames of
  // very different cost, and more resident work-groups hide the long ones.
  std::vector<Plan> rule(n_frames);
  size_t rule_bp = 0, rule_fp = 0;
  const Tuning by_rule{0, 0, 0, {0, 0, 0}};
  int32_t segs[8];
  const int nseg = fwd_seg_candidates(segs, 8);
  for (int i = 0; i < n_frames; ++i) {
    std::string m;
    pa_status st = make_plan(&frames[i], dtype, &rule[i], &m, &by_rule);
    for (int c = nseg - 1; st == PA_OK && rule[i].fp_lds > kLdsBatchFwd && c >= 0; --c) {
      if (segs[c] >= rule[i].op.fseg) continue;
      Plan shorter;
      const Tuning t{segs[c], 0, 0, {0, 0, 0}};
      if (make_plan(&frames[i], dtype, &shorter, &m, &t) == PA_OK && shorter.op.fseg == segs[c])
        rule[i] = shorter;
    }
    if (st != PA_OK) {
      if (msg) *msg = "frame " + std::to_string(i) + ": " + m;
      return st;
    }
    if (i > 0 && frames[i].ndim != frames[0].ndim)
      return fail(msg, PA_ERR_INVALID_ARGUMENT, "every frame of a batch must have the same ndim");
    rule_bp = std::max(rule_bp, rule[i].bp_lds);
    rule_fp = std::max(rule_fp, rule[i].fp_lds);
  }
  for (int i = 0; i < n_frames; ++i) {
    std::string m;
    Plan tuned;
    if (use_tuning && make_plan(&frames[i], dtype, &tuned, &m) == PA_OK && tuned.bp_lds <= rule_bp &&
        tuned.fp_lds <= rule_fp && tuned.op.ffix == rule[i].op.ffix)
      B.plans[i] = tuned;
    else
      B.plans[i] = rule[i];
  }
  for (Plan& pl : B.plans) pl.two_pass = false;   // batched launches use the sensor-major forward
  B.tuned = use_tuning;
  B.ffix = B.plans[0].op.ffix != 0;   // one forward kernel per launch: every frame plans the same mode
  B.ndim = frames[0].ndim;
  B.elem = B.plans[0].elem;
  // packed buffers in caller order
  B.xoff.assign(n_frames + 1, 0);
  B.yoff.assign(n_frames + 1, 0);
  for (int i = 0; i < n_frames; ++i) {
    B.xoff[i + 1] = B.xoff[i] + B.plans[i].P;
    B.yoff[i + 1] = B.yoff[i] + B.plans[i].M;
  }
  B.P_total = B.xoff[n_frames];
  B.M_total = B.yoff[n_frames];
  if (B.P_total > std::numeric_limits<int32_t>::max() || B.M_total > std::numeric_limits<int32_t>::max() * 4ll)
    return fail(msg, PA_ERR_UNSUPPORTED, "packed batch too large");
  // largest frames first, so the long work-groups start early (stable for ties)
  std::vector<int> order(n_frames);
  for (int i = 0; i < n_frames; ++i) order[i] = i;
  auto work = [&](int i) { return (double)B.plans[i].P * (double)B.plans[i].op.S; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  int64_t bbp = 0, bfp = 0, bm = 0, bpp = 0, sbp = 0, sfp = 0;
  B.table.resize(n_frames);
  for (int j = 0; j < n_frames; ++j) {
    const int i = order[j];
    const Plan& pl = B.plans[i];
    FrameDesc& F = B.table[j];
    std::memset(&F, 0, sizeof(F));
    F.op = pl.op;
    F.frame = i;
    F.xo = B.xoff[i];
    F.yo = B.yoff[i];
    F.b_bp = (int32_t)bbp; F.n_bp = pl.bp_grid; bbp += F.n_bp;
    F.b_fp = (int32_t)bfp; F.n_fp = pl.fp_grid; bfp += F.n_fp;
    F.b_m = (int32_t)bm; F.n_m = blas_grid(pl.M); bm += F.n_m;
    F.b_p = (int32_t)bpp; F.n_p = blas_grid(pl.P); bpp += F.n_p;
    F.s_bp = (int32_t)sbp; sbp += std::max(F.n_bp, 1);
    F.s_fp = (int32_t)sfp; sfp += std::max(F.n_fp, 1);
    B.frac = B.frac || pl.op.t0f != 0.0f;
    B.bp_lds = std::max(B.bp_lds, pl.bp_lds);
    B.fp_lds = std::max(B.fp_lds, pl.fp_lds);
  }
  const int64_t lim = std::numeric_limits<int32_t>::max();
  if (bbp > lim || bfp > lim || bm > lim || bpp > lim || sbp > lim || sfp > lim)
    return fail(msg, PA_ERR_UNSUPPORTED, "batch needs more than 2^31-1 work-groups in one launch");
  B.bp_grid = (int)bbp;
  B.fp_grid = (int)bfp;
  B.m_grid = (int)bm;
  B.p_grid = (int)bpp;
  B.bp_slots = (int)sbp;
  B.fp_slots = (int)sfp;
  *bp = std::move(B);
  return PA_OK;
}

BatchLayout batch_layout(const BatchPlan& B, int32_t iters, bool cg) {
  BatchLayout L{};
  const size_t A = 256;
  size_t off = 0;
  L.table = off; off = align_up(off + sizeof(FrameDesc) * (size_t)B.nf, A);
  if (!cg) {
    L.total = off;
    return L;
  }
  L.astride = std::max(iters, 0) + 2;
  const size_t nf = (size_t)B.nf;
  L.status = off; off = align_up(off + sizeof(int) * nf, A);
  L.gamma = off; off = align_up(off + sizeof(double) * nf * L.astride, A);
  L.alpha = off; off = align_up(off + sizeof(double) * nf * L.astride, A);
  L.part_q = off; off = align_up(off + sizeof(double) * B.fp_slots, A);
  L.part_r = off; off = align_up(off + sizeof(double) * B.m_grid, A);
  L.part_s = off; off = align_up(off + sizeof(double) * B.bp_slots, A);
  L.part_x = off; off = align_up(off + sizeof(double) * B.bp_slots, A);
  L.part_p = off; off = align_up(off + sizeof(double) * B.p_grid, A);
  L.vec_r = off; off = align_up(off + B.elem * (size_t)std::max<int64_t>(B.M_total, 1), A);
  L.vec_q = off; off = align_up(off + B.elem * (size_t)std::max<int64_t>(B.M_total, 1), A);
  L.vec_s = off; off = align_up(off + B.elem * (size_t)std::max<int64_t>(B.P_total, 1), A);
  L.vec_p = off; off = align_up(off + B.elem * (size_t)std::max<int64_t>(B.P_total, 1), A);
  L.total = off;
  return L;
}

}  // namespace pa
