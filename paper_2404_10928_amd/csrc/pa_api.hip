// The C ABI (include/pa.h): argument checks on the host, then kernel enqueues
// on the caller's stream.  The library allocates no device memory: the
// caller owns every buffer, including the CGLS workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <list>
#include <mutex>
#include <string>
#include <vector>
#include <new>

#include "pa.h"
#include "pa_dense.h"
#include "pa_freq.h"
#include "pa_kernels.h"
#include "pa_plan.h"

namespace {

thread_local std::string g_err;

pa_status set_err(pa_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

pa_status hip_err(hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return set_err(PA_ERR_HIP, m);
}

#define PA_HIP(call, where)                       \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_err(e_, where); \
  } while (0)

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + nb && b0 < a0 + na;
}

pa_status plan_or_fail(const pa_geometry* g, pa_dtype dt, pa::Plan* pl) {
  std::string msg;
  pa_status st = pa::make_plan(g, dt, pl, &msg);
  if (st != PA_OK) return set_err(st, msg);
  return PA_OK;
}

pa_status check_vec(const void* p, int64_t n, size_t elem, const char* name) {
  if (n > 0 && !p) return set_err(PA_ERR_INVALID_ARGUMENT, std::string(name) + " is NULL");
  if (p && !aligned(p, elem)) return set_err(PA_ERR_INVALID_ARGUMENT, std::string(name) + " is not aligned to its element size");
  return PA_OK;
}

// ---------------------------------------------------------------- CGLS enqueue

struct Solve {
  const pa::Plan* pl;
  pa::CglsLayout L;
  const void* y;
  void* x;
  int iters;
  double lambda;
  uint32_t flags;
  unsigned char* ws;
  double* hist;
};

hipError_t enqueue_cgls(const Solve& S, hipStream_t st) {
  const pa::Plan& pl = *S.pl;
  const pa::CglsLayout& L = S.L;
  const pa_dtype dt = pl.dtype;
  unsigned char* ws = S.ws;
  int* status = reinterpret_cast<int*>(ws + L.status);
  double* gamma = reinterpret_cast<double*>(ws + L.gamma);
  double* alpha = reinterpret_cast<double*>(ws + L.alpha);
  double* part_q = reinterpret_cast<double*>(ws + L.part_q);
  double* part_r = reinterpret_cast<double*>(ws + L.part_r);
  double* part_s = reinterpret_cast<double*>(ws + L.part_s);
  double* part_x = reinterpret_cast<double*>(ws + L.part_x);
  double* part_p = reinterpret_cast<double*>(ws + L.part_p);
  void* r = ws + L.vec_r;
  void* q = ws + L.vec_q;
  void* s = ws + L.vec_s;
  void* p = ws + L.vec_p;
  void* fwd = ws + L.fwd;   // partial rows of the forward operator (when its plan uses them)
  hipError_t e;
  const int gbp = std::max(pl.bp_grid, 1);

  // r0 = y - A x0 ; s0 = A^T r0 - lambda x0 ; p0 = s0
  if (S.flags & PA_X0_ZERO) {
    if ((e = pa::launch_fill(dt, S.x, pl.P, st)) != hipSuccess) return e;
    if ((e = pa::launch_init_r(dt, r, S.y, nullptr, pl.M, part_r, status, alpha, st)) != hipSuccess) return e;
  } else {
    if ((e = pa::launch_forward(pl, S.x, q, nullptr, fwd, st)) != hipSuccess) return e;
    if ((e = pa::launch_init_r(dt, r, S.y, q, pl.M, part_r, status, alpha, st)) != hipSuccess) return e;
  }
  pa::CgArgs cg{S.x, p, alpha, S.lambda, part_s, part_x};
  auto adjoint_cg = [&](const double* a) -> hipError_t {
    if (pl.bp_grid == 0) {  // no pixels: nothing to update, the sums are zero
      hipError_t ee = pa::launch_fill(PA_F64, part_s, gbp, st);
      if (ee != hipSuccess) return ee;
      return pa::launch_fill(PA_F64, part_x, gbp, st);
    }
    pa::CgArgs c2 = cg;
    c2.alpha = a;
    return pa::launch_adjoint(pl, r, s, &c2, st);
  };
  if ((e = adjoint_cg(alpha)) != hipSuccess) return e;
  if (L.fused) {
    // The direction update p_k = s_k + beta p_{k-1} (with gamma[k], history
    // row k and the partials of ||p_k||^2) rides on pass 1 of q = A p_k; p_k
    // alternates between two buffers.  The last history row comes from the
    // direction kernel with no vector to update.
    void* pb[2] = {p, ws + L.vec_p2};
    for (int k = 0; k < S.iters; ++k) {
      pa::CgDirArgs d{};
      d.s = static_cast<const float*>(s);
      d.p_old = static_cast<const float*>(pb[(k + 1) & 1]);
      d.p_new = static_cast<float*>(pb[k & 1]);
      d.part_s = part_s;
      d.part_x = part_x;
      d.part_r = part_r;
      d.gs = gbp;
      d.gx = gbp;
      d.gr = L.g_m;
      d.lambda = S.lambda;
      d.gamma = gamma;
      d.status = status;
      d.hist = S.hist;
      d.part_p = part_p;
      d.k = k;
      if ((e = pa::launch_forward_cg(pl, d, static_cast<float*>(q), part_q, fwd, st)) != hipSuccess) return e;
      if ((e = pa::launch_upd_r(dt, r, q, pl.M, part_q, L.g_q, part_p, L.g_pf, S.lambda, gamma + k, alpha + k + 1,
                                status, k, part_r, st)) != hipSuccess)
        return e;
      cg.p = pb[k & 1];
      if ((e = adjoint_cg(alpha + k + 1)) != hipSuccess) return e;
    }
    return pa::launch_dir(dt, nullptr, s, 0, nullptr, 0, part_s, gbp, part_x, gbp, part_r, L.g_m, S.lambda, gamma,
                          S.iters - 1, status, S.hist, part_p, st);
  }
  if ((e = pa::launch_dir(dt, p, s, pl.P, nullptr, 0, part_s, gbp, part_x, gbp, part_r, L.g_m, S.lambda, gamma, -1,
                          status, S.hist, part_p, st)) != hipSuccess)
    return e;
  for (int k = 0; k < S.iters; ++k) {
    // q = A p with the FP64 partials of ||q||^2
    if ((e = pa::launch_forward(pl, p, q, part_q, fwd, st)) != hipSuccess) return e;
    if ((e = pa::launch_upd_r(dt, r, q, pl.M, part_q, L.g_q, part_p, L.g_p, S.lambda, gamma + k, alpha + k + 1, status,
                              k, part_r, st)) != hipSuccess)
      return e;
    if ((e = adjoint_cg(alpha + k + 1)) != hipSuccess) return e;
    if ((e = pa::launch_dir(dt, p, s, pl.P, nullptr, 0, part_s, gbp, part_x, gbp, part_r, L.g_m, S.lambda, gamma, k,
                            status, S.hist, part_p, st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------- Landweber enqueue

struct LwSolve {
  const pa::Plan* pl;
  pa::LwLayout L;
  const void* y;
  void* x;
  int iters;
  double lambda;
  double omega;      // > 0: given; 0: estimated by power iteration
  int power_iters;
  uint32_t flags;
  unsigned char* ws;
  double* hist;
};

hipError_t enqueue_landweber(const LwSolve& S, hipStream_t st) {
  const pa::Plan& pl = *S.pl;
  const pa::LwLayout& L = S.L;
  const pa_dtype dt = pl.dtype;
  unsigned char* ws = S.ws;
  int* status = reinterpret_cast<int*>(ws + L.status);
  double* alpha0 = reinterpret_cast<double*>(ws + L.alpha0);
  double* sigma2 = reinterpret_cast<double*>(ws + L.sigma2);
  double* omega = reinterpret_cast<double*>(ws + L.omega);
  double* part_r = reinterpret_cast<double*>(ws + L.part_r);
  double* part_s = reinterpret_cast<double*>(ws + L.part_s);
  double* part_x = reinterpret_cast<double*>(ws + L.part_x);
  double* part_n = reinterpret_cast<double*>(ws + L.part_n);
  void* r = ws + L.vec_r;
  void* q = ws + L.vec_q;
  void* s = ws + L.vec_s;
  void* v = ws + L.vec_v;
  void* fwd = ws + L.fwd;
  hipError_t e;
  // step size
  if ((e = pa::launch_fill(PA_F64, sigma2, 1, st)) != hipSuccess) return e;
  if (!(S.omega > 0.0) && pl.P > 0) {
    if ((e = pa::launch_fill_value(dt, v, pl.P, 1.0 / std::sqrt((double)pl.P), st)) != hipSuccess) return e;
    for (int it = 0; it < S.power_iters; ++it) {
      if ((e = pa::launch_forward(pl, v, q, nullptr, fwd, st)) != hipSuccess) return e;
      if (pl.bp_grid > 0 && (e = pa::launch_adjoint(pl, q, s, nullptr, st)) != hipSuccess) return e;
      if ((e = pa::launch_norm2(dt, s, pl.P, part_n, st)) != hipSuccess) return e;
      if ((e = pa::launch_pw_scale(dt, v, s, pl.P, part_n, sigma2, st)) != hipSuccess) return e;
    }
  }
  if ((e = pa::launch_pw_omega(sigma2, S.lambda, S.omega, omega, st)) != hipSuccess) return e;
  if (S.flags & PA_X0_ZERO)
    if ((e = pa::launch_fill(dt, S.x, pl.P, st)) != hipSuccess) return e;
  const int gbp = std::max(pl.bp_grid, 1);
  // s = A^T r - lambda x with x unchanged (the epilogue's step is the zero that init_r writes)
  pa::CgArgs cg{S.x, S.x, alpha0, S.lambda, part_s, part_x};
  for (int k = 0; k < S.iters; ++k) {
    if ((e = pa::launch_forward(pl, S.x, q, nullptr, fwd, st)) != hipSuccess) return e;
    if ((e = pa::launch_init_r(dt, r, S.y, q, pl.M, part_r, status, alpha0, st)) != hipSuccess) return e;
    if (pl.bp_grid == 0) {
      if ((e = pa::launch_fill(PA_F64, part_s, gbp, st)) != hipSuccess) return e;
      if ((e = pa::launch_fill(PA_F64, part_x, gbp, st)) != hipSuccess) return e;
    } else if ((e = pa::launch_adjoint(pl, r, s, &cg, st)) != hipSuccess) {
      return e;
    }
    if ((e = pa::launch_lw_step(dt, S.x, s, pl.P, part_r, L.g_m, part_x, gbp, S.lambda, omega, S.hist, k, st)) !=
        hipSuccess)
      return e;
  }
  // F at the final iterate
  if ((e = pa::launch_forward(pl, S.x, q, nullptr, fwd, st)) != hipSuccess) return e;
  if ((e = pa::launch_init_r(dt, r, S.y, q, pl.M, part_r, status, alpha0, st)) != hipSuccess) return e;
  if ((e = pa::launch_norm2(dt, S.x, pl.P, part_n, st)) != hipSuccess) return e;
  return pa::launch_lw_final(part_r, L.g_m, part_n, L.g_p, S.lambda, S.hist, S.iters, st);
}

// ------------------------------------------ proximal gradient (FISTA) enqueue

struct FiSolve {
  const pa::Plan* pl;
  pa::FistaLayout F;
  int nx, ny;
  const void* y;
  void* x;
  int iters;
  double lambda, alpha, beta, eps;
  double omega;      // > 0: given; 0: estimated by power iteration
  int power_iters;
  uint32_t flags;
  unsigned char* ws;
  double* hist;
};

hipError_t enqueue_fista(const FiSolve& S, hipStream_t st) {
  const pa::Plan& pl = *S.pl;
  const pa::LwLayout& L = S.F.lw;
  const pa_dtype dt = pl.dtype;
  unsigned char* ws = S.ws;
  int* status = reinterpret_cast<int*>(ws + L.status);
  double* alpha0 = reinterpret_cast<double*>(ws + L.alpha0);
  double* sigma2 = reinterpret_cast<double*>(ws + L.sigma2);
  double* omega = reinterpret_cast<double*>(ws + L.omega);
  double* part_r = reinterpret_cast<double*>(ws + L.part_r);
  double* part_s = reinterpret_cast<double*>(ws + L.part_s);
  double* part_x = reinterpret_cast<double*>(ws + L.part_x);
  double* part_n = reinterpret_cast<double*>(ws + L.part_n);
  double* part_tv = reinterpret_cast<double*>(ws + S.F.part_tv);
  double* part_l1 = reinterpret_cast<double*>(ws + S.F.part_l1);
  void* r = ws + L.vec_r;
  void* q = ws + L.vec_q;
  void* s = ws + L.vec_s;
  void* v = ws + L.vec_v;
  void* zb[2] = {ws + S.F.vec_z0, ws + S.F.vec_z1};
  void* fwd = ws + L.fwd;
  const int nonneg = (S.flags & PA_NONNEG) ? 1 : 0;
  hipError_t e;
  // step: 1 / (sigma2 + lambda + 4 beta / eps), the inverse Lipschitz constant
  // of the smooth part's half-gradient (8 / eps bounds the TV Hessian)
  if ((e = pa::launch_fill(PA_F64, sigma2, 1, st)) != hipSuccess) return e;
  if (!(S.omega > 0.0) && pl.P > 0) {
    if ((e = pa::launch_fill_value(dt, v, pl.P, 1.0 / std::sqrt((double)pl.P), st)) != hipSuccess) return e;
    for (int it = 0; it < S.power_iters; ++it) {
      if ((e = pa::launch_forward(pl, v, q, nullptr, fwd, st)) != hipSuccess) return e;
      if (pl.bp_grid > 0 && (e = pa::launch_adjoint(pl, q, s, nullptr, st)) != hipSuccess) return e;
      if ((e = pa::launch_norm2(dt, s, pl.P, part_n, st)) != hipSuccess) return e;
      if ((e = pa::launch_pw_scale(dt, v, s, pl.P, part_n, sigma2, st)) != hipSuccess) return e;
    }
  }
  const double tv_l = S.beta > 0.0 ? 4.0 * S.beta / S.eps : 0.0;
  if ((e = pa::launch_pw_omega(sigma2, S.lambda + tv_l, S.omega, omega, st)) != hipSuccess) return e;
  if ((e = pa::launch_fill(dt, S.x, pl.P, st)) != hipSuccess) return e;
  if ((e = pa::launch_fill(dt, zb[0], pl.P, st)) != hipSuccess) return e;
  const int gbp = std::max(pl.bp_grid, 1);
  double t = 1.0;
  for (int k = 0; k < S.iters; ++k) {
    void* z = zb[k & 1];
    void* zn = zb[(k + 1) & 1];
    // r = y - A z ; s = A^T r - lambda z with the partials of ||z||^2 (the
    // epilogue's step is the zero that init_r writes, so z is unchanged)
    if ((e = pa::launch_forward(pl, z, q, nullptr, fwd, st)) != hipSuccess) return e;
    if ((e = pa::launch_init_r(dt, r, S.y, q, pl.M, part_r, status, alpha0, st)) != hipSuccess) return e;
    if (pl.bp_grid == 0) {
      if ((e = pa::launch_fill(PA_F64, part_s, gbp, st)) != hipSuccess) return e;
      if ((e = pa::launch_fill(PA_F64, part_x, gbp, st)) != hipSuccess) return e;
    } else {
      pa::CgArgs cg{z, z, alpha0, S.lambda, part_s, part_x};
      if ((e = pa::launch_adjoint(pl, r, s, &cg, st)) != hipSuccess) return e;
    }
    const double t1 = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    const double mu = (t - 1.0) / t1;
    if ((e = pa::launch_fista_step(dt, z, s, S.x, zn, S.nx, S.ny, pl.P, S.beta, S.eps, S.alpha, omega, mu, nonneg,
                                   part_tv, part_l1, st)) != hipSuccess)
      return e;
    if ((e = pa::launch_fista_hist(part_r, L.g_m, part_x, gbp, part_tv, part_l1, L.g_p, S.lambda, S.beta, S.alpha,
                                   S.hist, k, st)) != hipSuccess)
      return e;
    t = t1;
  }
  // the objective at the final iterate
  if ((e = pa::launch_forward(pl, S.x, q, nullptr, fwd, st)) != hipSuccess) return e;
  if ((e = pa::launch_init_r(dt, r, S.y, q, pl.M, part_r, status, alpha0, st)) != hipSuccess) return e;
  if ((e = pa::launch_fista_terms(dt, S.x, S.nx, S.ny, pl.P, S.beta, S.eps, part_n, part_tv, part_l1, st)) !=
      hipSuccess)
    return e;
  return pa::launch_fista_hist(part_r, L.g_m, part_n, L.g_p, part_tv, part_l1, L.g_p, S.lambda, S.beta, S.alpha,
                               S.hist, S.iters, st);
}

// ------------------------------------------------------------ graph cache

struct GraphKey {
  uint64_t batch;   // 0 for single-frame solves, else the batch's id (renewed whenever its plan changes)
  uint64_t epoch;   // single-frame solves: the tuning table's epoch the plan was made under
  pa_geometry g;
  pa_dtype dt;
  const void* y;
  void* x;
  int iters;
  double lambda;
  uint32_t flags;
  void* ws;
  double* hist;
  int device;
  int kind;           // 0 CGLS, 1 Landweber, 2 FISTA
  double omega;       // Landweber, FISTA: given step (0: estimated)
  int power_iters;    // Landweber, FISTA: power-iteration steps
  double alpha, beta, eps;  // FISTA: l1 weight, TV weight, TV smoothing
  bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
};

std::mutex g_graph_mu;
std::list<GraphEntry>* g_graphs = nullptr;  // never destroyed: graphs live until process exit
constexpr size_t kMaxGraphs = 16;
hipStream_t g_capture_stream[64] = {};

template <typename Enqueue>
hipError_t get_graph(const GraphKey& key, Enqueue&& enqueue, hipGraphExec_t* out) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  if (!g_graphs) g_graphs = new std::list<GraphEntry>();
  for (auto it = g_graphs->begin(); it != g_graphs->end(); ++it) {
    if (it->key == key) {
      g_graphs->splice(g_graphs->begin(), *g_graphs, it);
      *out = g_graphs->front().exec;
      return hipSuccess;
    }
  }
  hipError_t e;
  if (key.device < 0 || key.device >= 64) return hipErrorInvalidDevice;
  hipStream_t& cs = g_capture_stream[key.device];
  if (!cs && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return e;
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  hipError_t ee = enqueue(cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  if (ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return ee;
  }
  if (e != hipSuccess) return e;
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  if (g_graphs->size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(g_graphs->back().exec);
    g_graphs->pop_back();
  }
  g_graphs->push_front(GraphEntry{key, exec});
  *out = exec;
  return hipSuccess;
}

}  // namespace

// ------------------------------------------------------------------ batches

struct pa_batch {
  pa::BatchPlan plan;
  std::vector<pa_geometry> frames;   // the caller's geometries (device sensor pointers are theirs)
  pa::FrameDesc* pinned = nullptr;   // page-locked copy of plan.table (allocated on first use)
  uint64_t id = 0;
  std::mutex mu;
};

namespace {

std::atomic<uint64_t> g_batch_ids{1};

pa::BatchLaunch batch_launch(const pa::BatchPlan& B, unsigned char* ws, const pa::BatchLayout& L) {
  pa::BatchLaunch bl{};
  bl.table = reinterpret_cast<const pa::FrameDesc*>(ws + L.table);
  bl.nf = B.nf;
  bl.dtype = B.dtype;
  bl.ndim = B.ndim;
  bl.frac = B.frac;
  bl.ffix = B.ffix;
  bl.bp_grid = B.bp_grid;
  bl.fp_grid = B.fp_grid;
  bl.m_grid = B.m_grid;
  bl.p_grid = B.p_grid;
  bl.bp_lds = B.bp_lds;
  bl.fp_lds = B.fp_lds;
  bl.P_total = B.P_total;
  bl.M_total = B.M_total;
  return bl;
}

// Copies the frame table into the workspace (ordered on the stream before the
// work that reads it).
pa_status upload_table(pa_batch* b, unsigned char* ws, const pa::BatchLayout& L, hipStream_t st) {
  std::lock_guard<std::mutex> lk(b->mu);
  const size_t bytes = sizeof(pa::FrameDesc) * (size_t)b->plan.nf;
  if (!b->pinned) {
    void* h = nullptr;
    PA_HIP(hipHostMalloc(&h, bytes, hipHostMallocDefault), "hipHostMalloc (frame table)");
    std::memcpy(h, b->plan.table.data(), bytes);
    b->pinned = static_cast<pa::FrameDesc*>(h);
  }
  PA_HIP(hipMemcpyAsync(ws + L.table, b->pinned, bytes, hipMemcpyHostToDevice, st), "frame table upload");
  return PA_OK;
}

pa_status check_batch_ws(const pa_batch* b, const void* ws, size_t bytes, const pa::BatchLayout& L) {
  if (!b) return set_err(PA_ERR_INVALID_ARGUMENT, "batch is NULL");
  if (!ws) return set_err(PA_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(ws, 256)) return set_err(PA_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (bytes < L.total) return set_err(PA_ERR_WORKSPACE, "workspace smaller than the size pa_batch_*workspace_bytes() gives");
  return PA_OK;
}

pa_status check_batch_vecs(const pa_batch* b, const void* x, const void* y, const void* ws, size_t wsb) {
  const pa::BatchPlan& B = b->plan;
  pa_status st;
  if ((st = check_vec(x, B.P_total, B.elem, "x")) != PA_OK) return st;
  if ((st = check_vec(y, B.M_total, B.elem, "y")) != PA_OK) return st;
  if (overlap(x, B.P_total * B.elem, y, B.M_total * B.elem)) return set_err(PA_ERR_INVALID_ARGUMENT, "x and y overlap");
  if (overlap(ws, wsb, x, B.P_total * B.elem) || overlap(ws, wsb, y, B.M_total * B.elem))
    return set_err(PA_ERR_INVALID_ARGUMENT, "workspace overlaps x or y");
  return PA_OK;
}

struct BatchSolve {
  const pa::BatchPlan* B;
  pa::BatchLayout L;
  const void* y;
  void* x;
  int iters;
  double lambda;
  uint32_t flags;
  unsigned char* ws;
  double* hist;
};

// The batched CGLS: the single-frame sequence of launches, each covering
// every frame, with per-frame scalars.
hipError_t enqueue_batch_cgls(const BatchSolve& S, hipStream_t st) {
  const pa::BatchPlan& B = *S.B;
  const pa::BatchLayout& L = S.L;
  unsigned char* ws = S.ws;
  const pa::BatchLaunch bl = batch_launch(B, ws, L);
  int* status = reinterpret_cast<int*>(ws + L.status);
  double* gamma = reinterpret_cast<double*>(ws + L.gamma);
  double* alpha = reinterpret_cast<double*>(ws + L.alpha);
  double* part_q = reinterpret_cast<double*>(ws + L.part_q);
  double* part_r = reinterpret_cast<double*>(ws + L.part_r);
  double* part_s = reinterpret_cast<double*>(ws + L.part_s);
  double* part_x = reinterpret_cast<double*>(ws + L.part_x);
  double* part_p = reinterpret_cast<double*>(ws + L.part_p);
  void* r = ws + L.vec_r;
  void* q = ws + L.vec_q;
  void* s = ws + L.vec_s;
  void* p = ws + L.vec_p;
  const int as = L.astride;
  const int hs = 3 * (S.iters + 1);
  hipError_t e;
  // slots of frames without adjoint or forward work stay zero for the whole solve
  if ((e = pa::launch_fill(PA_F64, part_s, B.bp_slots, st)) != hipSuccess) return e;
  if ((e = pa::launch_fill(PA_F64, part_x, B.bp_slots, st)) != hipSuccess) return e;
  if ((e = pa::launch_fill(PA_F64, part_q, B.fp_slots, st)) != hipSuccess) return e;
  if (S.flags & PA_X0_ZERO) {
    if ((e = pa::launch_fill(B.dtype, S.x, B.P_total, st)) != hipSuccess) return e;
    if ((e = pa::launch_init_r_batched(bl, r, S.y, nullptr, part_r, status, alpha, as, st)) != hipSuccess) return e;
  } else {
    if ((e = pa::launch_forward_batched(bl, S.x, q, nullptr, st)) != hipSuccess) return e;
    if ((e = pa::launch_init_r_batched(bl, r, S.y, q, part_r, status, alpha, as, st)) != hipSuccess) return e;
  }
  pa::BatchCg cg{S.x, p, alpha, as, 0, S.lambda, part_s, part_x};
  if ((e = pa::launch_adjoint_batched(bl, r, s, &cg, st)) != hipSuccess) return e;
  if ((e = pa::launch_dir_batched(bl, p, s, part_s, part_x, part_r, S.lambda, gamma, as, -1, status, S.hist, hs, part_p,
                                  st)) != hipSuccess)
    return e;
  for (int k = 0; k < S.iters; ++k) {
    if ((e = pa::launch_forward_batched(bl, p, q, part_q, st)) != hipSuccess) return e;
    if ((e = pa::launch_upd_r_batched(bl, r, q, part_q, part_p, S.lambda, gamma, alpha, as, status, k, part_r, st)) !=
        hipSuccess)
      return e;
    cg.acol = k + 1;
    if ((e = pa::launch_adjoint_batched(bl, r, s, &cg, st)) != hipSuccess) return e;
    if ((e = pa::launch_dir_batched(bl, p, s, part_s, part_x, part_r, S.lambda, gamma, as, k, status, S.hist, hs,
                                    part_p, st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

int32_t pa_abi_version(void) { return PA_ABI_VERSION; }

const char* pa_last_error(void) { return g_err.c_str(); }

pa_status pa_validate_geometry(const pa_geometry* g, pa_dtype dtype) {
  g_err.clear();
  pa::Plan pl;
  return plan_or_fail(g, dtype, &pl);
}

pa_status pa_forward(const pa_geometry* g, pa_dtype dtype, const void* x, void* y, void* hip_stream) {
  g_err.clear();
  pa::Plan pl;
  pa_status st = plan_or_fail(g, dtype, &pl);
  if (st != PA_OK) return st;
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  if ((st = check_vec(y, pl.M, pl.elem, "y")) != PA_OK) return st;
  if (overlap(x, pl.P * pl.elem, y, pl.M * pl.elem)) return set_err(PA_ERR_INVALID_ARGUMENT, "x and y overlap");
  PA_HIP(pa::launch_forward(pl, x, y, nullptr, nullptr, static_cast<hipStream_t>(hip_stream)), "forward kernel");
  return PA_OK;
}

// The scratch of pa_forward_noalloc: a device array that every GPU the
// library runs on holds until the process ends.  In host code `scratch`
// names a host-side stand-in, not device memory: host code uses only the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[PA_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kScratchDevices];   // per device: device address of `scratch`, looked up once

pa_status noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_err(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices) return set_err(PA_ERR_UNSUPPORTED, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_err(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_err(PA_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return PA_OK;
}
}  // namespace

pa_status pa_forward_noalloc(const pa_geometry* g, pa_dtype dtype, const void* x, void* y, void* hip_stream) {
  g_err.clear();
  pa::Plan pl;
  pa_status st = plan_or_fail(g, dtype, &pl);
  if (st != PA_OK) return st;
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  if ((st = check_vec(y, pl.M, pl.elem, "y")) != PA_OK) return st;
  if (overlap(x, pl.P * pl.elem, y, pl.M * pl.elem)) return set_err(PA_ERR_INVALID_ARGUMENT, "x and y overlap");
  const size_t need = pl.two_pass ? pl.fwd_scratch : 0;
  if (need > PA_NOALLOC_SCRATCH_BYTES)
    return set_err(PA_ERR_UNSUPPORTED, "the planned forward needs " + std::to_string(need) +
                                           " bytes of scratch, above PA_NOALLOC_SCRATCH_BYTES (" +
                                           std::to_string((size_t)PA_NOALLOC_SCRATCH_BYTES) + ")");
  void* ws = nullptr;
  if (need > 0 && (st = noalloc_scratch(&ws)) != PA_OK) return st;
  PA_HIP(pa::launch_forward(pl, x, y, nullptr, ws, static_cast<hipStream_t>(hip_stream)), "forward kernels");
  return PA_OK;
}

size_t pa_forward_workspace_bytes(const pa_geometry* g, pa_dtype dtype) {
  g_err.clear();
  pa::Plan pl;
  if (plan_or_fail(g, dtype, &pl) != PA_OK) return 0;
  return pl.two_pass ? pl.fwd_scratch : 0;
}

pa_status pa_forward_ws(const pa_geometry* g, pa_dtype dtype, const void* x, void* y, void* workspace,
                        size_t workspace_bytes, void* hip_stream) {
  g_err.clear();
  pa::Plan pl;
  pa_status st = plan_or_fail(g, dtype, &pl);
  if (st != PA_OK) return st;
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  if ((st = check_vec(y, pl.M, pl.elem, "y")) != PA_OK) return st;
  if (overlap(x, pl.P * pl.elem, y, pl.M * pl.elem)) return set_err(PA_ERR_INVALID_ARGUMENT, "x and y overlap");
  const size_t need = pl.two_pass ? pl.fwd_scratch : 0;
  if (need > 0) {
    if (!workspace) return set_err(PA_ERR_WORKSPACE, "workspace is NULL");
    if (!aligned(workspace, 256)) return set_err(PA_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    if (workspace_bytes < need) return set_err(PA_ERR_WORKSPACE, "workspace smaller than pa_forward_workspace_bytes()");
    if (overlap(workspace, need, x, pl.P * pl.elem) || overlap(workspace, need, y, pl.M * pl.elem))
      return set_err(PA_ERR_INVALID_ARGUMENT, "workspace overlaps x or y");
  }
  PA_HIP(pa::launch_forward(pl, x, y, nullptr, need > 0 ? workspace : nullptr, static_cast<hipStream_t>(hip_stream)),
         "forward kernels");
  return PA_OK;
}

pa_status pa_adjoint(const pa_geometry* g, pa_dtype dtype, const void* y, void* x, void* hip_stream) {
  g_err.clear();
  pa::Plan pl;
  pa_status st = plan_or_fail(g, dtype, &pl);
  if (st != PA_OK) return st;
  if ((st = check_vec(y, pl.M, pl.elem, "y")) != PA_OK) return st;
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  if (overlap(x, pl.P * pl.elem, y, pl.M * pl.elem)) return set_err(PA_ERR_INVALID_ARGUMENT, "x and y overlap");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  PA_HIP(pa::launch_adjoint(pl, y, x, nullptr, s), "adjoint kernel");
  return PA_OK;
}

size_t pa_cgls_workspace_bytes(const pa_geometry* g, pa_dtype dtype, int32_t iters) {
  g_err.clear();
  if (iters < 0) {
    set_err(PA_ERR_INVALID_ARGUMENT, "iters must be >= 0");
    return 0;
  }
  pa::Plan pl;
  if (plan_or_fail(g, dtype, &pl) != PA_OK) return 0;
  return pa::cgls_layout(pl, iters).total;
}

pa_status pa_cgls_solve(const pa_geometry* g, pa_dtype dtype, const void* y, void* x, int32_t iters, double lambda,
                        uint32_t flags, void* workspace, size_t workspace_bytes, double* history, void* hip_stream) {
  g_err.clear();
  const uint64_t epoch = pa::tune_epoch();  // read before planning: a later tuning makes a new key
  pa::Plan pl;
  pa_status st = plan_or_fail(g, dtype, &pl);
  if (st != PA_OK) return st;
  if (iters < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "iters must be >= 0");
  if (iters > (1 << 20)) return set_err(PA_ERR_UNSUPPORTED, "iters above 2^20");
  if (!std::isfinite(lambda) || lambda < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "lambda must be finite and >= 0");
  if (flags & ~(PA_X0_ZERO | PA_USE_GRAPH)) return set_err(PA_ERR_INVALID_ARGUMENT, "unknown flag bits");
  if ((st = check_vec(y, pl.M, pl.elem, "y")) != PA_OK) return st;
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  if (history && !aligned(history, 8)) return set_err(PA_ERR_INVALID_ARGUMENT, "history is not 8-byte aligned");
  const pa::CglsLayout L = pa::cgls_layout(pl, iters);
  if (!workspace) return set_err(PA_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(workspace, 256)) return set_err(PA_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (workspace_bytes < L.total) return set_err(PA_ERR_WORKSPACE, "workspace smaller than pa_cgls_workspace_bytes()");
  if (overlap(x, pl.P * pl.elem, y, pl.M * pl.elem)) return set_err(PA_ERR_INVALID_ARGUMENT, "x and y overlap");
  if (overlap(workspace, L.total, x, pl.P * pl.elem) || overlap(workspace, L.total, y, pl.M * pl.elem))
    return set_err(PA_ERR_INVALID_ARGUMENT, "workspace overlaps x or y");
  if (history && (overlap(history, sizeof(double) * 3 * (size_t)(iters + 1), workspace, L.total) ||
                  overlap(history, sizeof(double) * 3 * (size_t)(iters + 1), x, pl.P * pl.elem) ||
                  overlap(history, sizeof(double) * 3 * (size_t)(iters + 1), y, pl.M * pl.elem)))
    return set_err(PA_ERR_INVALID_ARGUMENT, "history overlaps another buffer");

  Solve S{&pl, L, y, x, iters, lambda, flags, static_cast<unsigned char*>(workspace), history};
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  bool use_graph = (flags & PA_USE_GRAPH) != 0;
  if (use_graph && s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    PA_HIP(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) use_graph = false;  // already inside the caller's capture
  }
  if (!use_graph) {
    PA_HIP(enqueue_cgls(S, s), "CGLS enqueue");
    return PA_OK;
  }
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.g = *g;
  key.epoch = epoch;
  key.dt = dtype;
  key.y = y;
  key.x = x;
  key.iters = iters;
  key.lambda = lambda;
  key.flags = flags;
  key.ws = workspace;
  key.hist = history;
  PA_HIP(hipGetDevice(&key.device), "hipGetDevice");
  hipGraphExec_t exec = nullptr;
  PA_HIP(get_graph(key, [&](hipStream_t cs) { return enqueue_cgls(S, cs); }, &exec), "CGLS graph capture");
  PA_HIP(hipGraphLaunch(exec, s), "hipGraphLaunch");
  return PA_OK;
}

pa_status pa_cgls_stop_iteration(const void* workspace, int32_t* stop_iter) {
  g_err.clear();
  if (!workspace || !stop_iter) return set_err(PA_ERR_INVALID_ARGUMENT, "NULL argument");
  int v = -1;
  PA_HIP(hipMemcpy(&v, workspace, sizeof(int), hipMemcpyDeviceToHost), "read CGLS status");
  *stop_iter = v;
  return v >= 0 ? PA_ERR_BREAKDOWN : PA_OK;
}

pa_status pa_batch_create(const pa_geometry* frames, int32_t n_frames, pa_dtype dtype, pa_batch** out) {
  g_err.clear();
  if (!out) return set_err(PA_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  pa::BatchPlan B;
  std::string msg;
  pa_status st = pa::make_batch_plan(frames, n_frames, dtype, &B, &msg);
  if (st != PA_OK) return set_err(st, msg);
  pa_batch* b = new (std::nothrow) pa_batch();
  if (!b) return set_err(PA_ERR_INVALID_ARGUMENT, "out of host memory");
  b->plan = std::move(B);
  b->frames.assign(frames, frames + n_frames);
  b->id = g_batch_ids.fetch_add(1);
  *out = b;
  return PA_OK;
}

size_t pa_batch_autotune_workspace_bytes(const pa_batch* b) {
  g_err.clear();
  if (!b) {
    set_err(PA_ERR_INVALID_ARGUMENT, "batch is NULL");
    return 0;
  }
  size_t n = 0;
  for (int c = 0; c < 2; ++c) {
    pa::BatchPlan B;
    std::string msg;
    if (pa::make_batch_plan(b->frames.data(), (int32_t)b->frames.size(), b->plan.dtype, &B, &msg, c == 1) != PA_OK) {
      set_err(PA_ERR_INVALID_ARGUMENT, msg);
      return 0;
    }
    n = std::max(n, pa::batch_layout(B, 0, false).total);
  }
  return n;
}

pa_status pa_batch_autotune(pa_batch* b, void* x, void* y, void* workspace, size_t workspace_bytes,
                            void* hip_stream, int32_t* tuned) {
  g_err.clear();
  if (!b) return set_err(PA_ERR_INVALID_ARGUMENT, "batch is NULL");
  pa::BatchPlan cand[2];
  std::string msg;
  for (int c = 0; c < 2; ++c) {
    pa_status st = pa::make_batch_plan(b->frames.data(), (int32_t)b->frames.size(), b->plan.dtype, &cand[c], &msg,
                                       c == 1);
    if (st != PA_OK) return set_err(st, msg);
  }
  pa_status st;
  if ((st = check_batch_vecs(b, x, y, workspace, workspace_bytes)) != PA_OK) return st;
  if (!workspace || !aligned(workspace, 256)) return set_err(PA_ERR_WORKSPACE, "workspace is NULL or misaligned");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PA_HIP(hipEventCreate(&e0), "hipEventCreate");
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_err(he, "hipEventCreate");
  }
  float best = 3.0e38f;
  int pick = 0;
  hipError_t err = hipSuccess;
  for (int c = 0; c < 2 && err == hipSuccess; ++c) {
    const pa::BatchLayout L = pa::batch_layout(cand[c], 0, false);
    if (L.total > workspace_bytes) continue;  // this candidate needs a larger workspace
    const size_t tb = sizeof(pa::FrameDesc) * cand[c].table.size();
    // the table goes through a synchronous copy here (the stream is synchronised below anyway)
    if ((err = hipStreamSynchronize(s)) != hipSuccess) break;
    if ((err = hipMemcpy(ws + L.table, cand[c].table.data(), tb, hipMemcpyHostToDevice)) != hipSuccess) break;
    const pa::BatchLaunch bl = batch_launch(cand[c], ws, L);
    auto run = [&]() -> hipError_t {
      hipError_t e = pa::launch_forward_batched(bl, x, y, nullptr, s);
      if (e != hipSuccess) return e;
      return pa::launch_adjoint_batched(bl, y, x, nullptr, s);
    };
    if ((err = run()) != hipSuccess) break;
    float t = 3.0e38f;
    for (int trial = 0; trial < 3 && err == hipSuccess; ++trial) {
      if ((err = hipEventRecord(e0, s)) != hipSuccess) break;
      for (int r = 0; r < 3 && err == hipSuccess; ++r) err = run();
      if (err != hipSuccess) break;
      if ((err = hipEventRecord(e1, s)) != hipSuccess) break;
      if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
      float ms = 0.f;
      if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      t = std::min(t, ms);
    }
    if (err == hipSuccess && t < best) {
      best = t;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return hip_err(err, "batch autotune");
  if (best == 3.0e38f) return set_err(PA_ERR_WORKSPACE, "workspace too small for every candidate plan");
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->plan = std::move(cand[pick]);
    b->id = g_batch_ids.fetch_add(1);  // graphs captured under the old plan no longer match
    if (b->pinned) {
      (void)hipHostFree(b->pinned);
      b->pinned = nullptr;
    }
  }
  if (tuned) *tuned = pick;
  return PA_OK;
}

pa_status pa_batch_destroy(pa_batch* b) {
  g_err.clear();
  if (!b) return PA_OK;
  hipError_t e = hipSuccess;
  if (b->pinned) e = hipHostFree(b->pinned);
  delete b;
  if (e != hipSuccess) return hip_err(e, "hipHostFree (frame table)");
  return PA_OK;
}

pa_status pa_batch_offsets(const pa_batch* b, int64_t* x_offsets, int64_t* y_offsets) {
  g_err.clear();
  if (!b) return set_err(PA_ERR_INVALID_ARGUMENT, "batch is NULL");
  for (int i = 0; i <= b->plan.nf; ++i) {
    if (x_offsets) x_offsets[i] = b->plan.xoff[i];
    if (y_offsets) y_offsets[i] = b->plan.yoff[i];
  }
  return PA_OK;
}

size_t pa_batch_workspace_bytes(const pa_batch* b) {
  g_err.clear();
  if (!b) {
    set_err(PA_ERR_INVALID_ARGUMENT, "batch is NULL");
    return 0;
  }
  return pa::batch_layout(b->plan, 0, false).total;
}

size_t pa_batch_cgls_workspace_bytes(const pa_batch* b, int32_t iters) {
  g_err.clear();
  if (!b) {
    set_err(PA_ERR_INVALID_ARGUMENT, "batch is NULL");
    return 0;
  }
  if (iters < 0) {
    set_err(PA_ERR_INVALID_ARGUMENT, "iters must be >= 0");
    return 0;
  }
  return pa::batch_layout(b->plan, iters, true).total;
}

pa_status pa_batch_forward(pa_batch* b, const void* x, void* y, void* workspace, size_t workspace_bytes,
                           void* hip_stream) {
  g_err.clear();
  if (!b) return set_err(PA_ERR_INVALID_ARGUMENT, "batch is NULL");
  const pa::BatchLayout L = pa::batch_layout(b->plan, 0, false);
  pa_status st;
  if ((st = check_batch_ws(b, workspace, workspace_bytes, L)) != PA_OK) return st;
  if ((st = check_batch_vecs(b, x, y, workspace, L.total)) != PA_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  if ((st = upload_table(b, ws, L, s)) != PA_OK) return st;
  PA_HIP(pa::launch_forward_batched(batch_launch(b->plan, ws, L), x, y, nullptr, s), "batched forward kernels");
  return PA_OK;
}

pa_status pa_batch_adjoint(pa_batch* b, const void* y, void* x, void* workspace, size_t workspace_bytes,
                           void* hip_stream) {
  g_err.clear();
  if (!b) return set_err(PA_ERR_INVALID_ARGUMENT, "batch is NULL");
  const pa::BatchLayout L = pa::batch_layout(b->plan, 0, false);
  pa_status st;
  if ((st = check_batch_ws(b, workspace, workspace_bytes, L)) != PA_OK) return st;
  if ((st = check_batch_vecs(b, x, y, workspace, L.total)) != PA_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  if ((st = upload_table(b, ws, L, s)) != PA_OK) return st;
  PA_HIP(pa::launch_adjoint_batched(batch_launch(b->plan, ws, L), y, x, nullptr, s), "batched adjoint kernel");
  return PA_OK;
}

pa_status pa_batch_cgls_solve(pa_batch* b, const void* y, void* x, int32_t iters, double lambda, uint32_t flags,
                              void* workspace, size_t workspace_bytes, double* history, void* hip_stream) {
  g_err.clear();
  if (!b) return set_err(PA_ERR_INVALID_ARGUMENT, "batch is NULL");
  if (iters < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "iters must be >= 0");
  if (iters > (1 << 20)) return set_err(PA_ERR_UNSUPPORTED, "iters above 2^20");
  if (!std::isfinite(lambda) || lambda < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "lambda must be finite and >= 0");
  if (flags & ~(PA_X0_ZERO | PA_USE_GRAPH)) return set_err(PA_ERR_INVALID_ARGUMENT, "unknown flag bits");
  const pa::BatchLayout L = pa::batch_layout(b->plan, iters, true);
  pa_status st;
  if ((st = check_batch_ws(b, workspace, workspace_bytes, L)) != PA_OK) return st;
  if ((st = check_batch_vecs(b, x, y, workspace, L.total)) != PA_OK) return st;
  const size_t hbytes = sizeof(double) * 3 * (size_t)(iters + 1) * (size_t)b->plan.nf;
  if (history && !aligned(history, 8)) return set_err(PA_ERR_INVALID_ARGUMENT, "history is not 8-byte aligned");
  if (history && (overlap(history, hbytes, workspace, L.total) ||
                  overlap(history, hbytes, x, b->plan.P_total * b->plan.elem) ||
                  overlap(history, hbytes, y, b->plan.M_total * b->plan.elem)))
    return set_err(PA_ERR_INVALID_ARGUMENT, "history overlaps another buffer");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  if ((st = upload_table(b, ws, L, s)) != PA_OK) return st;
  BatchSolve S{&b->plan, L, y, x, iters, lambda, flags, ws, history};
  bool use_graph = (flags & PA_USE_GRAPH) != 0;
  if (use_graph && s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    PA_HIP(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) use_graph = false;
  }
  if (!use_graph) {
    PA_HIP(enqueue_batch_cgls(S, s), "batched CGLS enqueue");
    return PA_OK;
  }
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.batch = b->id;
  key.dt = b->plan.dtype;
  key.y = y;
  key.x = x;
  key.iters = iters;
  key.lambda = lambda;
  key.flags = flags;
  key.ws = workspace;
  key.hist = history;
  PA_HIP(hipGetDevice(&key.device), "hipGetDevice");
  hipGraphExec_t exec = nullptr;
  PA_HIP(get_graph(key, [&](hipStream_t cs) { return enqueue_batch_cgls(S, cs); }, &exec), "batched CGLS graph capture");
  PA_HIP(hipGraphLaunch(exec, s), "hipGraphLaunch");
  return PA_OK;
}

pa_status pa_batch_stop_iterations(const pa_batch* b, const void* workspace, int32_t iters, int32_t* stop) {
  g_err.clear();
  if (!b || !workspace || !stop) return set_err(PA_ERR_INVALID_ARGUMENT, "NULL argument");
  if (iters < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "iters must be >= 0");
  const pa::BatchLayout L = pa::batch_layout(b->plan, iters, true);
  std::vector<int> v((size_t)b->plan.nf, -1);
  PA_HIP(hipMemcpy(v.data(), static_cast<const unsigned char*>(workspace) + L.status, sizeof(int) * v.size(),
                   hipMemcpyDeviceToHost),
         "read batched CGLS status");
  bool any = false;
  for (int i = 0; i < b->plan.nf; ++i) {
    stop[i] = v[i];
    any = any || v[i] >= 0;
  }
  return any ? PA_ERR_BREAKDOWN : PA_OK;
}

size_t pa_autotune_workspace_bytes(const pa_geometry* g, pa_dtype dtype) {
  g_err.clear();
  pa::Plan base;
  if (plan_or_fail(g, dtype, &base) != PA_OK) return 0;
  size_t n = 0;
  if (dtype == PA_F32) {
    int cand[8][3];
    const int nc = pa::fwd_tile_candidates(base.ndim, cand, 8);
    for (int i = 0; i < nc; ++i) {
      pa::Tuning t{0, 0, 3, {cand[i][0], cand[i][1], cand[i][2]}};
      pa::Plan pl;
      std::string msg;
      if (pa::make_plan(g, dtype, &pl, &msg, &t) == PA_OK && pl.two_pass) n = std::max(n, pl.fwd_scratch);
    }
  }
  return n;
}

pa_status pa_autotune(const pa_geometry* g, pa_dtype dtype, void* x, void* y, void* workspace, size_t workspace_bytes,
                      void* hip_stream, pa_tuning* out) {
  g_err.clear();
  pa::Plan base;
  pa_status st = plan_or_fail(g, dtype, &base);
  if (st != PA_OK) return st;
  if ((st = check_vec(x, base.P, base.elem, "x")) != PA_OK) return st;
  if ((st = check_vec(y, base.M, base.elem, "y")) != PA_OK) return st;
  if (overlap(x, base.P * base.elem, y, base.M * base.elem)) return set_err(PA_ERR_INVALID_ARGUMENT, "x and y overlap");
  if (workspace && !aligned(workspace, 256)) return set_err(PA_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (workspace && (overlap(workspace, workspace_bytes, x, base.P * base.elem) ||
                    overlap(workspace, workspace_bytes, y, base.M * base.elem)))
    return set_err(PA_ERR_INVALID_ARGUMENT, "workspace overlaps x or y");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PA_HIP(hipEventCreate(&e0), "hipEventCreate");
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_err(he, "hipEventCreate");
  }
  // time per launch: the best of three runs of kReps back-to-back launches
  constexpr int kReps = 8;
  auto time_it = [&](auto&& launch, float* us) -> hipError_t {
    hipError_t e;
    if ((e = launch()) != hipSuccess) return e;  // warm-up (and first-use attribute setting)
    float best = 3.0e38f;
    for (int trial = 0; trial < 3; ++trial) {
      if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
      for (int r = 0; r < kReps; ++r)
        if ((e = launch()) != hipSuccess) return e;
      if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
      best = std::min(best, ms * 1000.f / kReps);
    }
    *us = best;
    return hipSuccess;
  };
  pa::Tuning best{0, 0, 0, {0, 0, 0}};
  float best_f = 3.0e38f, best_a = 3.0e38f;
  hipError_t err = hipSuccess;
  // the forward kernel skips all-zero tiles, so time it on a full image
  err = pa::launch_fill_value(dtype, x, base.P, 1.0, s);
  if (err == hipSuccess) err = pa::launch_fill_value(dtype, y, base.M, 1.0, s);
  // forward segment lengths (and, with FP32 delay arithmetic, both accumulation modes)
  if (base.fp_grid > 0 && err == hipSuccess) {
    int32_t cand[8];
    const int nc = pa::fwd_seg_candidates(cand, 8);
    const int nmode = dtype == PA_F64 ? 1 : 2;
    for (int mode = 1; mode <= nmode && err == hipSuccess; ++mode) {
      int last_seg = -1;
      for (int i = 0; i < nc && err == hipSuccess; ++i) {
        pa::Tuning t{cand[i], 0, dtype == PA_F64 ? 0 : mode, {0, 0, 0}};
        pa::Plan pl;
        std::string msg;
        if (pa::make_plan(g, dtype, &pl, &msg, &t) != PA_OK) continue;
        if (pl.op.fseg == last_seg) continue;  // clipped to the same segment as the previous candidate
        last_seg = pl.op.fseg;
        float us = 0.f;
        err = time_it([&] { return pa::launch_forward(pl, x, y, nullptr, nullptr, s); }, &us);
        if (err == hipSuccess && us < best_f) {
          best_f = us;
          best.fwd_seg = pl.op.fseg;
          best.fwd_mode = t.fwd_mode;
        }
      }
    }
    // the partial-row method (PA_F32), for forward tiles whose rows fit the workspace
    if (dtype == PA_F32 && workspace) {
      int tc[8][3];
      const int ntc = pa::fwd_tile_candidates(base.ndim, tc, 8);
      for (int i = 0; i < ntc && err == hipSuccess; ++i) {
        pa::Tuning t{0, 0, 3, {tc[i][0], tc[i][1], tc[i][2]}};
        pa::Plan pl;
        std::string msg;
        if (pa::make_plan(g, dtype, &pl, &msg, &t) != PA_OK || !pl.two_pass) continue;
        if (pl.op.msub[0] != tc[i][0] || pl.op.msub[1] != tc[i][1] || pl.op.msub[2] != tc[i][2]) continue;
        if (pl.fwd_scratch > workspace_bytes) continue;
        float us = 0.f;
        err = time_it([&] { return pa::launch_forward(pl, x, y, nullptr, workspace, s); }, &us);
        if (err == hipSuccess && us < best_f) {
          best_f = us;
          best.fwd_seg = pl.op.fseg;
          best.fwd_mode = 3;
          for (int a = 0; a < 3; ++a) best.fwd_tile[a] = tc[i][a];
        }
      }
    }
  }
  // adjoint LDS budgets
  if (base.bp_grid > 0 && err == hipSuccess) {
    size_t cand[8];
    const int nc = pa::adj_lds_candidates(cand, 8);
    int last_sc = -1;
    for (int i = 0; i < nc && err == hipSuccess; ++i) {
      pa::Tuning t{0, (int32_t)cand[i], 0, {0, 0, 0}};
      pa::Plan pl;
      std::string msg;
      if (pa::make_plan(g, dtype, &pl, &msg, &t) != PA_OK) continue;
      if (pl.op.sc == last_sc) continue;  // same sensor chunk as the previous budget
      last_sc = pl.op.sc;
      float us = 0.f;
      err = time_it([&] { return pa::launch_adjoint(pl, y, x, nullptr, s); }, &us);
      if (err == hipSuccess && us < best_a) {
        best_a = us;
        best.adj_lds = t.adj_lds;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return hip_err(err, "autotune");
  pa::tune_store(g, dtype, best);
  if (out) {
    out->fwd_seg = best.fwd_seg;
    out->fwd_mode = best.fwd_mode;
    for (int a = 0; a < 3; ++a) out->fwd_tile[a] = best.fwd_tile[a];
    out->adj_lds_bytes = best.adj_lds;
    out->fwd_us = best_f < 3.0e38f ? best_f : 0.0;
    out->adj_us = best_a < 3.0e38f ? best_a : 0.0;
  }
  return PA_OK;
}

pa_status pa_tuning_set(const pa_geometry* g, pa_dtype dtype, const pa_tuning* t) {
  g_err.clear();
  if (!t) return set_err(PA_ERR_INVALID_ARGUMENT, "tuning pointer is NULL");
  pa::Plan base;
  pa_status st = plan_or_fail(g, dtype, &base);
  if (st != PA_OK) return st;
  if (t->fwd_seg < 0 || t->adj_lds_bytes < 0 || t->fwd_mode < 0 || t->fwd_mode > 3)
    return set_err(PA_ERR_INVALID_ARGUMENT, "fwd_seg, adj_lds_bytes >= 0 and fwd_mode in 0..3 required");
  if (t->fwd_mode == 3) {
    if (dtype != PA_F32) return set_err(PA_ERR_UNSUPPORTED, "fwd_mode 3 (partial rows) is PA_F32 only");
    for (int a = 0; a < 3; ++a)
      if (t->fwd_tile[a] < 1) return set_err(PA_ERR_INVALID_ARGUMENT, "fwd_mode 3 needs fwd_tile >= 1 on every axis");
  }
  if (t->fwd_mode == 2 && dtype == PA_F64) return set_err(PA_ERR_UNSUPPORTED, "PA_F64 has fwd_mode 0 only");
  pa::Tuning tu{t->fwd_seg, t->adj_lds_bytes, t->fwd_mode, {t->fwd_tile[0], t->fwd_tile[1], t->fwd_tile[2]}};
  pa::Plan pl;
  std::string msg;
  if ((st = pa::make_plan(g, dtype, &pl, &msg, &tu)) != PA_OK) return set_err(st, msg);
  // every requested choice must be the one the planner takes
  if (t->fwd_seg > 0 && pl.fp_grid > 0 && pl.op.fseg != std::min<int32_t>(t->fwd_seg, g->n_samples))
    return set_err(PA_ERR_UNSUPPORTED, "fwd_seg: the forward histogram does not fit in LDS");
  if (t->fwd_mode == 3 && (!pl.two_pass || pl.op.msub[0] != t->fwd_tile[0] || pl.op.msub[1] != t->fwd_tile[1] ||
                           pl.op.msub[2] != t->fwd_tile[2]))
    return set_err(PA_ERR_UNSUPPORTED, "fwd_tile: the partial-row tile does not fit this geometry");
  pa::tune_store(g, dtype, tu);
  return PA_OK;
}

pa_status pa_tuning_clear(void) {
  g_err.clear();
  pa::tune_clear();
  return PA_OK;
}

size_t pa_landweber_workspace_bytes(const pa_geometry* g, pa_dtype dtype) {
  g_err.clear();
  pa::Plan pl;
  if (plan_or_fail(g, dtype, &pl) != PA_OK) return 0;
  return pa::lw_layout(pl).total;
}

pa_status pa_landweber_solve(const pa_geometry* g, pa_dtype dtype, const void* y, void* x, int32_t iters,
                             double lambda, double omega, int32_t power_iters, uint32_t flags, void* workspace,
                             size_t workspace_bytes, double* history, void* hip_stream) {
  g_err.clear();
  const uint64_t epoch = pa::tune_epoch();  // read before planning: a later tuning makes a new key
  pa::Plan pl;
  pa_status st = plan_or_fail(g, dtype, &pl);
  if (st != PA_OK) return st;
  if (iters < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "iters must be >= 0");
  if (iters > (1 << 20) || power_iters > (1 << 20)) return set_err(PA_ERR_UNSUPPORTED, "iteration count above 2^20");
  if (!std::isfinite(lambda) || lambda < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "lambda must be finite and >= 0");
  if (!std::isfinite(omega) || omega < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "omega must be finite and >= 0");
  if (omega == 0.0 && power_iters < 1)
    return set_err(PA_ERR_INVALID_ARGUMENT, "omega == 0 needs power_iters >= 1 to estimate the step");
  if (flags & ~(PA_X0_ZERO | PA_USE_GRAPH)) return set_err(PA_ERR_INVALID_ARGUMENT, "unknown flag bits");
  if ((st = check_vec(y, pl.M, pl.elem, "y")) != PA_OK) return st;
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  if (history && !aligned(history, 8)) return set_err(PA_ERR_INVALID_ARGUMENT, "history is not 8-byte aligned");
  const pa::LwLayout L = pa::lw_layout(pl);
  if (!workspace) return set_err(PA_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(workspace, 256)) return set_err(PA_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (workspace_bytes < L.total) return set_err(PA_ERR_WORKSPACE, "workspace smaller than pa_landweber_workspace_bytes()");
  if (overlap(x, pl.P * pl.elem, y, pl.M * pl.elem)) return set_err(PA_ERR_INVALID_ARGUMENT, "x and y overlap");
  if (overlap(workspace, L.total, x, pl.P * pl.elem) || overlap(workspace, L.total, y, pl.M * pl.elem))
    return set_err(PA_ERR_INVALID_ARGUMENT, "workspace overlaps x or y");
  const size_t hb = sizeof(double) * (size_t)(iters + 1);
  if (history && (overlap(history, hb, workspace, L.total) || overlap(history, hb, x, pl.P * pl.elem) ||
                  overlap(history, hb, y, pl.M * pl.elem)))
    return set_err(PA_ERR_INVALID_ARGUMENT, "history overlaps another buffer");
  LwSolve S{&pl, L, y, x, iters, lambda, omega, omega > 0.0 ? 0 : power_iters, flags,
            static_cast<unsigned char*>(workspace), history};
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  bool use_graph = (flags & PA_USE_GRAPH) != 0;
  if (use_graph && s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    PA_HIP(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) use_graph = false;
  }
  if (!use_graph) {
    PA_HIP(enqueue_landweber(S, s), "Landweber enqueue");
    return PA_OK;
  }
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.g = *g;
  key.epoch = epoch;
  key.dt = dtype;
  key.y = y;
  key.x = x;
  key.iters = iters;
  key.lambda = lambda;
  key.flags = flags;
  key.ws = workspace;
  key.hist = history;
  key.kind = 1;
  key.omega = omega;
  key.power_iters = S.power_iters;
  PA_HIP(hipGetDevice(&key.device), "hipGetDevice");
  hipGraphExec_t exec = nullptr;
  PA_HIP(get_graph(key, [&](hipStream_t cs) { return enqueue_landweber(S, cs); }, &exec), "Landweber graph capture");
  PA_HIP(hipGraphLaunch(exec, s), "hipGraphLaunch");
  return PA_OK;
}

pa_status pa_landweber_step(const void* workspace, double* omega, double* sigma2) {
  g_err.clear();
  if (!workspace) return set_err(PA_ERR_INVALID_ARGUMENT, "workspace is NULL");
  double v[3] = {0, 0, 0};  // sigma2, omega follow alpha0 in the layout
  PA_HIP(hipMemcpy(v, static_cast<const unsigned char*>(workspace) + 64, sizeof(v), hipMemcpyDeviceToHost),
         "read Landweber step");
  if (sigma2) *sigma2 = v[1];
  if (omega) *omega = v[2];
  return PA_OK;
}

size_t pa_fista_workspace_bytes(const pa_geometry* g, pa_dtype dtype) {
  g_err.clear();
  pa::Plan pl;
  if (plan_or_fail(g, dtype, &pl) != PA_OK) return 0;
  return pa::fista_layout(pl).total;
}

pa_status pa_fista_solve(const pa_geometry* g, pa_dtype dtype, const void* y, void* x, int32_t iters, double lambda,
                         double alpha, double beta, double eps, double omega, int32_t power_iters, uint32_t flags,
                         void* workspace, size_t workspace_bytes, double* history, void* hip_stream) {
  g_err.clear();
  const uint64_t epoch = pa::tune_epoch();  // read before planning: a later tuning makes a new key
  pa::Plan pl;
  pa_status st = plan_or_fail(g, dtype, &pl);
  if (st != PA_OK) return st;
  if (iters < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "iters must be >= 0");
  if (iters > (1 << 20) || power_iters > (1 << 20)) return set_err(PA_ERR_UNSUPPORTED, "iteration count above 2^20");
  if (!std::isfinite(lambda) || lambda < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "lambda must be finite and >= 0");
  if (!std::isfinite(alpha) || alpha < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "alpha must be finite and >= 0");
  if (!std::isfinite(beta) || beta < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "beta must be finite and >= 0");
  if (beta > 0) {
    if (!std::isfinite(eps) || !(eps > 0)) return set_err(PA_ERR_INVALID_ARGUMENT, "eps must be finite and > 0");
    if (g->ndim != 2 || g->nz != 1) return set_err(PA_ERR_UNSUPPORTED, "the TV term (beta > 0) needs a 2D image");
  }
  if (!std::isfinite(omega) || omega < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "omega must be finite and >= 0");
  if (omega == 0.0 && power_iters < 1)
    return set_err(PA_ERR_INVALID_ARGUMENT, "omega == 0 needs power_iters >= 1 to estimate the step");
  if (flags & ~(PA_NONNEG | PA_USE_GRAPH)) return set_err(PA_ERR_INVALID_ARGUMENT, "unknown flag bits");
  if ((st = check_vec(y, pl.M, pl.elem, "y")) != PA_OK) return st;
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  if (history && !aligned(history, 8)) return set_err(PA_ERR_INVALID_ARGUMENT, "history is not 8-byte aligned");
  const pa::FistaLayout F = pa::fista_layout(pl);
  if (!workspace) return set_err(PA_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(workspace, 256)) return set_err(PA_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (workspace_bytes < F.total) return set_err(PA_ERR_WORKSPACE, "workspace smaller than pa_fista_workspace_bytes()");
  if (overlap(x, pl.P * pl.elem, y, pl.M * pl.elem)) return set_err(PA_ERR_INVALID_ARGUMENT, "x and y overlap");
  if (overlap(workspace, F.total, x, pl.P * pl.elem) || overlap(workspace, F.total, y, pl.M * pl.elem))
    return set_err(PA_ERR_INVALID_ARGUMENT, "workspace overlaps x or y");
  const size_t hb = sizeof(double) * (size_t)(iters + 1);
  if (history && (overlap(history, hb, workspace, F.total) || overlap(history, hb, x, pl.P * pl.elem) ||
                  overlap(history, hb, y, pl.M * pl.elem)))
    return set_err(PA_ERR_INVALID_ARGUMENT, "history overlaps another buffer");
  FiSolve S{&pl, F, g->nx, g->ny, y, x, iters, lambda, alpha, beta, beta > 0 ? eps : 1.0,
            omega, omega > 0.0 ? 0 : power_iters, flags, static_cast<unsigned char*>(workspace), history};
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  bool use_graph = (flags & PA_USE_GRAPH) != 0;
  if (use_graph && s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    PA_HIP(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) use_graph = false;
  }
  if (!use_graph) {
    PA_HIP(enqueue_fista(S, s), "FISTA enqueue");
    return PA_OK;
  }
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.g = *g;
  key.epoch = epoch;
  key.dt = dtype;
  key.y = y;
  key.x = x;
  key.iters = iters;
  key.lambda = lambda;
  key.flags = flags;
  key.ws = workspace;
  key.hist = history;
  key.kind = 2;
  key.omega = omega;
  key.power_iters = S.power_iters;
  key.alpha = alpha;
  key.beta = beta;
  key.eps = S.eps;
  PA_HIP(hipGetDevice(&key.device), "hipGetDevice");
  hipGraphExec_t exec = nullptr;
  PA_HIP(get_graph(key, [&](hipStream_t cs) { return enqueue_fista(S, cs); }, &exec), "FISTA graph capture");
  PA_HIP(hipGraphLaunch(exec, s), "hipGraphLaunch");
  return PA_OK;
}

pa_status pa_fista_step(const void* workspace, double* omega, double* sigma2) {
  // the FISTA layout keeps the Landweber fields at the same offsets
  return pa_landweber_step(workspace, omega, sigma2);
}

// ------------------------------------------------------ dense matrix path

namespace {
constexpr size_t kDenseMax = size_t(1) << 40;

// Validates g (as the operators do) and sets *bytes to the matrix size.
pa_status dense_bytes(const pa_geometry* g, pa_dtype dtype, pa::Plan* pl, size_t* bytes) {
  *bytes = 0;
  if (dtype == PA_MIXED) return set_err(PA_ERR_UNSUPPORTED, "the dense matrix path takes PA_F32 or PA_F64");
  pa_status st = plan_or_fail(g, dtype, pl);
  if (st != PA_OK) return st;
  const double n = (double)pl->M * (double)pa::dense_ld(pl->P) * (double)pl->elem;
  if (n > (double)kDenseMax) return set_err(PA_ERR_UNSUPPORTED, "dense matrix above 2^40 bytes");
  *bytes = std::max<size_t>((size_t)pl->M * (size_t)pa::dense_ld(pl->P) * pl->elem, 1);
  return PA_OK;
}
}  // namespace

size_t pa_dense_matrix_bytes(const pa_geometry* g, pa_dtype dtype) {
  g_err.clear();
  pa::Plan pl;
  size_t n = 0;
  return dense_bytes(g, dtype, &pl, &n) == PA_OK ? n : 0;
}

size_t pa_dense_adjoint_workspace_bytes(const pa_geometry* g, pa_dtype dtype) {
  g_err.clear();
  pa::Plan pl;
  size_t n = 0;
  if (dense_bytes(g, dtype, &pl, &n) != PA_OK) return 0;
  const pa::DenseShape s = pa::dense_shape(pl.P, pl.M);
  return std::max<size_t>(sizeof(double) * (size_t)s.nchunks * (size_t)s.ld, 256);
}

pa_status pa_dense_build(const pa_geometry* g, pa_dtype dtype, void* matrix, size_t matrix_bytes, void* hip_stream) {
  g_err.clear();
  pa::Plan pl;
  size_t need = 0;
  pa_status st = dense_bytes(g, dtype, &pl, &need);
  if (st != PA_OK) return st;
  if (!matrix) return set_err(PA_ERR_INVALID_ARGUMENT, "matrix is NULL");
  if (!aligned(matrix, 16)) return set_err(PA_ERR_INVALID_ARGUMENT, "matrix is not 16-byte aligned");
  if (matrix_bytes < need) return set_err(PA_ERR_WORKSPACE, "matrix smaller than pa_dense_matrix_bytes()");
  PA_HIP(pa::launch_dense_build(g, dtype, matrix, static_cast<hipStream_t>(hip_stream)), "dense build");
  return PA_OK;
}

pa_status pa_dense_forward(const pa_geometry* g, pa_dtype dtype, const void* matrix, size_t matrix_bytes,
                           const void* x, void* y, void* hip_stream) {
  g_err.clear();
  pa::Plan pl;
  size_t need = 0;
  pa_status st = dense_bytes(g, dtype, &pl, &need);
  if (st != PA_OK) return st;
  if (!matrix) return set_err(PA_ERR_INVALID_ARGUMENT, "matrix is NULL");
  if (!aligned(matrix, 16)) return set_err(PA_ERR_INVALID_ARGUMENT, "matrix is not 16-byte aligned");
  if (matrix_bytes < need) return set_err(PA_ERR_WORKSPACE, "matrix smaller than pa_dense_matrix_bytes()");
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  if ((st = check_vec(y, pl.M, pl.elem, "y")) != PA_OK) return st;
  if (pl.P > 0 && !aligned(x, 16)) return set_err(PA_ERR_INVALID_ARGUMENT, "x is not 16-byte aligned");
  if (overlap(x, pl.P * pl.elem, y, pl.M * pl.elem) || overlap(matrix, need, y, pl.M * pl.elem))
    return set_err(PA_ERR_INVALID_ARGUMENT, "y overlaps x or the matrix");
  PA_HIP(pa::launch_dense_forward(g, dtype, matrix, x, y, static_cast<hipStream_t>(hip_stream)), "dense forward");
  return PA_OK;
}

pa_status pa_dense_adjoint(const pa_geometry* g, pa_dtype dtype, const void* matrix, size_t matrix_bytes,
                           const void* y, void* x, void* workspace, size_t workspace_bytes, void* hip_stream) {
  g_err.clear();
  pa::Plan pl;
  size_t need = 0;
  pa_status st = dense_bytes(g, dtype, &pl, &need);
  if (st != PA_OK) return st;
  if (!matrix) return set_err(PA_ERR_INVALID_ARGUMENT, "matrix is NULL");
  if (!aligned(matrix, 16)) return set_err(PA_ERR_INVALID_ARGUMENT, "matrix is not 16-byte aligned");
  if (matrix_bytes < need) return set_err(PA_ERR_WORKSPACE, "matrix smaller than pa_dense_matrix_bytes()");
  if ((st = check_vec(y, pl.M, pl.elem, "y")) != PA_OK) return st;
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  const pa::DenseShape sh = pa::dense_shape(pl.P, pl.M);
  const size_t wneed = std::max<size_t>(sizeof(double) * (size_t)sh.nchunks * (size_t)sh.ld, 256);
  if (!workspace) return set_err(PA_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(workspace, 256)) return set_err(PA_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (workspace_bytes < wneed) return set_err(PA_ERR_WORKSPACE, "workspace smaller than pa_dense_adjoint_workspace_bytes()");
  if (overlap(x, pl.P * pl.elem, y, pl.M * pl.elem) || overlap(matrix, need, x, pl.P * pl.elem) ||
      overlap(workspace, wneed, x, pl.P * pl.elem) || overlap(workspace, wneed, matrix, need) ||
      overlap(workspace, wneed, y, pl.M * pl.elem))
    return set_err(PA_ERR_INVALID_ARGUMENT, "x, y, the matrix and the workspace must not overlap");
  PA_HIP(pa::launch_dense_adjoint(g, dtype, matrix, y, x, workspace, static_cast<hipStream_t>(hip_stream)),
         "dense adjoint");
  return PA_OK;
}

// ------------------------------------------------ frequency-domain operator

namespace {
pa_status freq_check(const pa_geometry* g, pa_dtype dtype, double f0, double df, int32_t nf, pa::Plan* pl) {
  if (dtype == PA_MIXED) return set_err(PA_ERR_UNSUPPORTED, "the frequency-domain operator takes PA_F32 or PA_F64");
  pa_status st = plan_or_fail(g, dtype, pl);
  if (st != PA_OK) return st;
  if (nf < 0 || nf > 65536) return set_err(PA_ERR_INVALID_ARGUMENT, "nf must be in [0, 65536]");
  if (!std::isfinite(f0) || f0 < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "f0 must be finite and >= 0");
  if (!std::isfinite(df) || df < 0) return set_err(PA_ERR_INVALID_ARGUMENT, "df must be finite and >= 0");
  return PA_OK;
}

pa_status freq_buffers(const pa::Plan& pl, int32_t nf, const void* x, const void* Y, void* workspace,
                       size_t workspace_bytes) {
  pa_status st;
  const int64_t ny = 2 * (int64_t)pl.op.S * nf;
  if ((st = check_vec(x, pl.P, pl.elem, "x")) != PA_OK) return st;
  if ((st = check_vec(Y, ny, pl.elem, "Y")) != PA_OK) return st;
  const size_t need = pa::freq_shape(pl.P, pl.op.S, nf).workspace;
  if (!workspace) return set_err(PA_ERR_WORKSPACE, "workspace is NULL");
  if (!aligned(workspace, 256)) return set_err(PA_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (workspace_bytes < need) return set_err(PA_ERR_WORKSPACE, "workspace smaller than pa_freq_workspace_bytes()");
  if (overlap(x, pl.P * pl.elem, Y, ny * pl.elem) || overlap(workspace, need, x, pl.P * pl.elem) ||
      overlap(workspace, need, Y, ny * pl.elem))
    return set_err(PA_ERR_INVALID_ARGUMENT, "x, Y and the workspace must not overlap");
  return PA_OK;
}
}  // namespace

size_t pa_freq_workspace_bytes(const pa_geometry* g, pa_dtype dtype, int32_t nf) {
  g_err.clear();
  pa::Plan pl;
  if (freq_check(g, dtype, 0.0, 0.0, nf, &pl) != PA_OK) return 0;
  return pa::freq_shape(pl.P, pl.op.S, nf).workspace;
}

pa_status pa_freq_forward(const pa_geometry* g, pa_dtype dtype, double f0, double df, int32_t nf, const void* x,
                          void* Y, void* workspace, size_t workspace_bytes, void* hip_stream) {
  g_err.clear();
  pa::Plan pl;
  pa_status st = freq_check(g, dtype, f0, df, nf, &pl);
  if (st != PA_OK) return st;
  if ((st = freq_buffers(pl, nf, x, Y, workspace, workspace_bytes)) != PA_OK) return st;
  PA_HIP(pa::launch_freq_forward(g, dtype, f0, df, nf, x, Y, workspace, static_cast<hipStream_t>(hip_stream)),
         "frequency-domain forward");
  return PA_OK;
}

pa_status pa_freq_adjoint(const pa_geometry* g, pa_dtype dtype, double f0, double df, int32_t nf, const void* Y,
                          void* x, void* workspace, size_t workspace_bytes, void* hip_stream) {
  g_err.clear();
  pa::Plan pl;
  pa_status st = freq_check(g, dtype, f0, df, nf, &pl);
  if (st != PA_OK) return st;
  if ((st = freq_buffers(pl, nf, x, Y, workspace, workspace_bytes)) != PA_OK) return st;
  PA_HIP(pa::launch_freq_adjoint(g, dtype, f0, df, nf, Y, x, workspace, static_cast<hipStream_t>(hip_stream)),
         "frequency-domain adjoint");
  return PA_OK;
}

}  // extern "C"
