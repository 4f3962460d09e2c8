/* pa.h -- matrix-free photoacoustic forward operator, its adjoint and a
 * regularised least-squares (CGLS) solve, on one AMD Instinct MI355X (gfx950).
 *
 * The operator is the paper's time-domain measurement matrix (Sec. "Principle
 * of Iterative Reconstruction", Eq. 6: measurements y = K theta, rows indexed
 * by (probe m, sample s), columns by pixel (i,j), entries a delta at the
 * arrival time |r_ij - r_m| / c) with the 1/R spreading of the Green's
 * function in Eq. 7 and a unit-peak linear hat standing for the delta on the
 * sample grid:
 *
 *   R_ps   = max(|r_p - r_s|, r_min)
 *   tau_ps = (R_ps / c - t0) / dt                       delay in samples
 *   (A x)[s,k]   = sum_p x_p * max(0, 1 - |k - tau_ps|) / R_ps,   k = 0..K-1
 *   (A^T y)[p]   = sum_s sum_k y[s,k] * max(0, 1 - |k - tau_ps|) / R_ps
 *
 * Taps falling outside 0..K-1 are dropped in both, so A^T is the exact
 * adjoint of A.  The solve minimises ||A x - y||^2 + lambda ||x||^2, the data
 * term of the paper's objective (Eq. 8) with a Tikhonov term, whose gradient
 * 2 A^T (A x - y) is the statement that takes 96.7 % of the paper's runtime
 * (Table 3).
 *
 * Conventions shared by every call
 *  - Units are SI: metres, seconds, metres per second.
 *  - Pixel (ix, iy, iz) sits at center + (i - (n - 1) / 2) * h on each axis.
 *  - Images are [nz][ny][nx] with ix fastest (nz = 1 in 2D); measurements are
 *    [S][K] with k fastest.  Both are dense and contiguous.
 *  - Device pointers are the caller's (e.g. torch tensors): the library never
 *    frees them.  They must be 16-byte aligned.  Inputs and outputs must not
 *    overlap.
 *  - Calls are asynchronous on the given HIP stream (NULL = the null stream):
 *    they return once the work is enqueued; results are valid after the
 *    caller synchronises that stream.  Outputs are overwritten, never
 *    accumulated into.
 *  - Argument and geometry errors are found on the host before anything is
 *    enqueued and need no GPU.  A failing call returns a non-zero status and
 *    leaves a message for pa_last_error(); it has enqueued nothing unless the
 *    status is PA_ERR_HIP.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PA_ABI_VERSION 2

typedef enum {
  PA_OK = 0,
  PA_ERR_INVALID_ARGUMENT = 1, /* null/misaligned pointer, bad size, non-finite or non-positive parameter */
  PA_ERR_UNSUPPORTED = 2,      /* valid but outside what the kernels handle (e.g. a trace window too long for LDS) */
  PA_ERR_WORKSPACE = 3,        /* workspace missing or smaller than pa_cgls_workspace_bytes() */
  PA_ERR_HIP = 4,              /* a HIP runtime call failed; pa_last_error() has its message */
  PA_ERR_BREAKDOWN = 5         /* CGLS stopped early: gamma == 0 (converged) or delta == 0 / non-finite */
} pa_status;

typedef enum {
  PA_F32 = 0,  /* x, y and the CGLS vectors are float; every inner product, norm, step size and the history are double on the GPU */
  PA_F64 = 1,  /* everything is double */
  PA_MIXED = 2 /* x, y, every vector and every sum are double; the per-pair delay and weight are formed in FP32
                  arithmetic as in PA_F32 (FP64 for sensors near the pixels), so the operator costs about what
                  PA_F32 does while nothing is rounded to float */
} pa_dtype;

typedef struct {
  int32_t ndim;            /* 2 or 3 */
  int32_t nx, ny, nz;      /* image size; nz must be 1 when ndim == 2; each >= 0 */
  double h;                /* pixel pitch [m], > 0 */
  double center[3];        /* position of the grid centre [m]; center[2] ignored in 2D */
  int32_t n_sensors;       /* S >= 0 */
  const double* sensors;   /* DEVICE pointer, [S][ndim] sensor positions [m]; may be NULL when S == 0 */
  int32_t n_samples;       /* K >= 0 */
  double dt;               /* sample interval [s], > 0 */
  double t0;               /* time of sample 0 [s] (sample k is at t0 + k dt) */
  double c;                /* speed of sound [m/s], > 0 */
  double r_min;            /* distance clamp [m], >= 0; 0 selects h / 2 */
} pa_geometry;

/* Flags for pa_cgls_solve. */
#define PA_X0_ZERO 1u   /* start from x0 = 0 and ignore the contents of x on entry */
#define PA_USE_GRAPH 2u /* enqueue the whole solve as one HIP graph (captured once per argument set, then replayed) */
#define PA_NONNEG 4u    /* pa_fista_solve only: constrain the image to x >= 0 */

/* Host-only check of a geometry: sizes, finiteness, and that the kernels can
 * tile it.  Touches no GPU state and dereferences no device pointer. */
pa_status pa_validate_geometry(const pa_geometry* g, pa_dtype dtype);

/* y := A x.  x: image (float for PA_F32, double for PA_F64); y: [S][K] of the
 * same type.  The time-domain operator of Eq. 6 as stated above. */
pa_status pa_forward(const pa_geometry* g, pa_dtype dtype, const void* x, void* y, void* hip_stream);

/* y := A x as pa_forward, with a caller-owned device workspace of
 * pa_forward_workspace_bytes() bytes (256-byte aligned; may be NULL when that
 * size is 0).  With PA_F32, once pa_autotune has chosen the partial-row method
 * for this shape, the operator runs in two passes through the workspace: pass
 * 1 scatters each forward tile's taps for 64 sensors into LDS rows, written to
 * the workspace; pass 2 adds each sensor's rows up.  Both methods form every
 * sum in a fixed order; they round differently (each within the same bound
 * of the exact operator).  Otherwise it is pa_forward. */
size_t pa_forward_workspace_bytes(const pa_geometry* g, pa_dtype dtype);
pa_status pa_forward_ws(const pa_geometry* g, pa_dtype dtype, const void* x, void* y, void* workspace,
                        size_t workspace_bytes, void* hip_stream);

/* For callers that cannot allocate device memory or hand over a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): pa_forward_ws with the library's own device scratch in place of
 * the caller's workspace.  The scratch is a static device array of
 * PA_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the
 * process ends; its address on the current device is looked up on the first
 * call there.  A shape whose planned forward needs more scratch than that
 * (pa_forward_workspace_bytes) is refused with PA_ERR_UNSUPPORTED before
 * anything is enqueued.  Nothing in the scratch has to start at zero: a call
 * reads only bytes it wrote itself.  Every call on one GPU shares that GPU's
 * one array, which keeps the last call's contents, so calls whose work
 * overlaps on one GPU (other streams, other threads) race: serialise them.
 * The current device must be the one x, y and hip_stream belong to.  Calls
 * no hipMalloc, hipFree or other allocating routine. */
#define PA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pa_status pa_forward_noalloc(const pa_geometry* g, pa_dtype dtype, const void* x, void* y, void* hip_stream);

/* x := A^T y, delay-and-interpolate back-projection: the exact adjoint of
 * pa_forward (the K^T products of Table 4). */
pa_status pa_adjoint(const pa_geometry* g, pa_dtype dtype, const void* y, void* x, void* hip_stream);

/* Device workspace (bytes) that pa_cgls_solve needs for this geometry, dtype
 * and iteration count.  0 means the arguments are invalid (see pa_last_error). */
size_t pa_cgls_workspace_bytes(const pa_geometry* g, pa_dtype dtype, int32_t iters);

/* CGLS on min ||A x - y||^2 + lambda ||x||^2 (the iterative reconstruction
 * loop of Table 3; Bjorck's CGLS form of CG on the shifted normal equations):
 *   r = y - A x0; s = A^T r - lambda x0; p = s; gamma = ||s||^2
 *   repeat iters times: q = A p; delta = ||q||^2 + lambda ||p||^2;
 *     alpha = gamma / delta; x += alpha p; r -= alpha q;
 *     s = A^T r - lambda x; beta = ||s||^2 / gamma; gamma = ||s||^2; p = s + beta p
 * y: [S][K] device; x: image, device, in = x0 (unless PA_X0_ZERO), out = x_iters.
 * lambda >= 0.  iters >= 0.  workspace: device, >= pa_cgls_workspace_bytes(),
 * 256-byte aligned, owned by the caller and reused freely between calls that
 * are not in flight at the same time.
 * history: device double [iters + 1][3] holding (||r_k||, ||s_k||,
 * ||r_k||^2 + lambda ||x_k||^2) per iteration, or NULL.
 * The step sizes are computed on the GPU, so nothing is copied to the host
 * during the solve.  If gamma or delta becomes 0 or non-finite at iteration k
 * the remaining steps leave x unchanged; pa_cgls_stop_iteration reports k. */
pa_status pa_cgls_solve(const pa_geometry* g, pa_dtype dtype, const void* y, void* x, int32_t iters,
                        double lambda, uint32_t flags, void* workspace, size_t workspace_bytes,
                        double* history, void* hip_stream);

/* After the solve's stream has been synchronised: *stop_iter = the iteration
 * at which CGLS stopped early, or -1 if it ran all iterations.  Returns PA_OK,
 * PA_ERR_BREAKDOWN when it stopped early, or an error.  Performs one blocking
 * device-to-host copy. */
pa_status pa_cgls_stop_iteration(const void* workspace, int32_t* stop_iter);

/* ------------------------------------------------------- gradient iteration
 * Landweber iteration on the same objective (the gradient loop of Experiment
 * 2 / Table 3, whose statement t1 = 2 K^T (K x - y) is the gradient of the
 * data term):
 *   x_{k+1} = x_k + omega (A^T (y - A x_k) - lambda x_k),   k = 0 .. iters-1
 * With omega > 0 the caller's step is used.  With omega == 0 the step is
 * omega = 1 / (sigma2 + lambda), where sigma2 estimates the largest
 * eigenvalue of A^T A by power_iters power-iteration steps from the all-ones
 * vector (v <- A^T A v / ||A^T A v||; sigma2 = ||A^T A v|| at the last step),
 * all on the GPU.
 * history: device double [iters + 1], F_k = ||y - A x_k||^2 + lambda ||x_k||^2
 * for k = 0 .. iters, or NULL.  Flags, workspace rules and errors as for
 * pa_cgls_solve; PA_X0_ZERO starts from 0. */
size_t pa_landweber_workspace_bytes(const pa_geometry* g, pa_dtype dtype);
pa_status pa_landweber_solve(const pa_geometry* g, pa_dtype dtype, const void* y, void* x, int32_t iters,
                             double lambda, double omega, int32_t power_iters, uint32_t flags, void* workspace,
                             size_t workspace_bytes, double* history, void* hip_stream);

/* After synchronising: the step the last solve on this workspace used, and
 * the eigenvalue estimate (0 when the step was given).  One blocking copy. */
pa_status pa_landweber_step(const void* workspace, double* omega, double* sigma2);

/* ------------------------------------------ sparsity-regularised objective
 * The compressed-sensing objective of Eq. 8 with both sparsifying transforms
 * taken as the identity, plus the Tikhonov term of the solvers above:
 *   F(x) = ||A x - y||^2 + lambda ||x||^2 + beta TV_eps(x) + alpha ||x||_1
 * TV_eps(x) = sum_p sqrt(dx_p^2 + dy_p^2 + eps^2) over forward differences of
 * the 2D image (zero past the last column and row): the smoothed isotropic
 * form of the TV penalty, whose gradient is the reweighted difference-matrix
 * term t2 of Table 3 with the weights applied per pixel.
 * Solved by the accelerated proximal gradient method (FISTA, Beck and
 * Teboulle 2009) from x_0 = z_0 = 0, t_0 = 1, for k = 0 .. iters-1:
 *   x_{k+1} = shrink(z_k + omega (A^T (y - A z_k) - lambda z_k - (beta/2) dTV(z_k)), omega alpha / 2)
 *   t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
 *   z_{k+1} = x_{k+1} + ((t_k - 1) / t_{k+1}) (x_{k+1} - x_k)
 * shrink(v, tau) = sign(v) max(|v| - tau, 0), or max(v - tau, 0) with
 * PA_NONNEG.  With omega > 0 the caller's step is used; with omega == 0 it is
 * 1 / (sigma2 + lambda + 4 beta / eps), sigma2 from power_iters
 * power-iteration steps as in pa_landweber_solve (the inverse Lipschitz
 * constant of the smooth part's half-gradient).
 * alpha, beta, lambda >= 0 and finite; beta > 0 needs eps > 0 and a 2D image
 * (PA_ERR_UNSUPPORTED otherwise); eps is ignored when beta == 0.
 * The solve always starts from 0: x is output only.  Flags: PA_NONNEG,
 * PA_USE_GRAPH.  history: device double [iters + 1] with F(z_k) for
 * k < iters (the objective at the point where the gradient is taken) and
 * F(x_iters) last, or NULL.  Vectors are FP32 under PA_F32 and FP64 under
 * PA_F64; every norm, TV sum and scalar is FP64 on the GPU.  Workspace rules
 * and errors as for pa_cgls_solve; pa_fista_step reads the step used. */
size_t pa_fista_workspace_bytes(const pa_geometry* g, pa_dtype dtype);
pa_status pa_fista_solve(const pa_geometry* g, pa_dtype dtype, const void* y, void* x, int32_t iters, double lambda,
                         double alpha, double beta, double eps, double omega, int32_t power_iters, uint32_t flags,
                         void* workspace, size_t workspace_bytes, double* history, void* hip_stream);

/* After synchronising: the step the last FISTA solve on this workspace used
 * and the eigenvalue estimate (0 when the step was given).  One blocking copy. */
pa_status pa_fista_step(const void* workspace, double* omega, double* sigma2);

/* ------------------------------------------------------ dense matrix path
 * The paper's own formulation (Experiment 2): the time-domain measurement
 * matrix kn materialised densely and applied as kn * x and kn' * y (the
 * statement that takes 96.7 % of Table 3).  The entries are those of
 * pa_forward: A[m][p] = (1/R_ps) max(0, 1 - |k - tau_ps|) for m = s * K + k,
 * formed in FP64 and rounded once to the dtype.  Rows are ld = P rounded up
 * to a multiple of 32 apart (padding columns are zero), so the matrix takes
 * pa_dense_matrix_bytes() = S * K * ld * sizeof(element) bytes of device
 * memory, owned by the caller (8.6 GB in FP64 for a 128 x 128 image, 128
 * sensors and 512 samples).  Both products accumulate in FP64 in a fixed
 * order and are bound by HBM bandwidth: each reads the whole matrix.
 * Returns 0 from the size queries when the arguments are invalid or the
 * matrix would exceed 2^40 bytes. */
size_t pa_dense_matrix_bytes(const pa_geometry* g, pa_dtype dtype);
/* A := the dense matrix of g (device, >= pa_dense_matrix_bytes(), 16-byte aligned). */
pa_status pa_dense_build(const pa_geometry* g, pa_dtype dtype, void* matrix, size_t matrix_bytes, void* hip_stream);
/* y := A x with a matrix pa_dense_build wrote for the same geometry and dtype. */
pa_status pa_dense_forward(const pa_geometry* g, pa_dtype dtype, const void* matrix, size_t matrix_bytes,
                           const void* x, void* y, void* hip_stream);
/* x := A^T y; workspace (device, caller-owned, 256-byte aligned) holds the FP64
 * partial sums of row chunks. */
size_t pa_dense_adjoint_workspace_bytes(const pa_geometry* g, pa_dtype dtype);
pa_status pa_dense_adjoint(const pa_geometry* g, pa_dtype dtype, const void* matrix, size_t matrix_bytes,
                           const void* y, void* x, void* workspace, size_t workspace_bytes, void* hip_stream);

/* ------------------------------------------------ frequency-domain operator
 * The frequency-domain measurement matrix of Eq. 7, matrix-free:
 *   K(s, n)_p = i c k_n exp(-i k_n R_ps) / R_ps,  k_n = 2 pi f_n / c,  f_n = f0 + n df,
 * n = 0 .. nf-1, with R_ps clamped at r_min as in pa_forward (the geometry's
 * dt, t0 and n_samples are not used).  Y is complex, stored as interleaved
 * (re, im) pairs [S][nf][2] of the dtype.
 *   pa_freq_forward: Y := K x for a real image x.
 *   pa_freq_adjoint: x := Re(K^H Y), the adjoint for the real inner product
 *   sum Re(Y) Re(Z) + Im(Y) Im(Z).
 * The phase f_n R / c is formed and reduced in FP64, the sine and cosine are
 * taken in the dtype, and every sum is FP64 in a fixed order (partial sums in
 * the caller's workspace, >= pa_freq_workspace_bytes(), 256-byte aligned).
 * f0, df >= 0 and finite; 0 <= nf <= 65536.  Returns 0 from the size query on
 * invalid arguments. */
size_t pa_freq_workspace_bytes(const pa_geometry* g, pa_dtype dtype, int32_t nf);
pa_status pa_freq_forward(const pa_geometry* g, pa_dtype dtype, double f0, double df, int32_t nf, const void* x,
                          void* Y, void* workspace, size_t workspace_bytes, void* hip_stream);
pa_status pa_freq_adjoint(const pa_geometry* g, pa_dtype dtype, double f0, double df, int32_t nf, const void* Y,
                          void* x, void* workspace, size_t workspace_bytes, void* hip_stream);

/* ------------------------------------------------------------------ batches
 * Many frames of uneven image size, sensor count and trace length, each with
 * its own geometry, processed by one launch per step.  Frame i's image and
 * traces sit in packed buffers at the element offsets pa_batch_offsets()
 * gives (the frames one after another, in the order passed to
 * pa_batch_create).  The batched kernels run the single-frame device code on
 * each frame's own plan and form every partial sum in the same order, so a
 * frame's result is the same, bit for bit, as that frame batched on its own,
 * and as a single-frame call under the same plan.  Batched launches use the
 * sensor-major forward (no workspace).  Their planner keeps each frame's
 * forward LDS within 48 KiB (shorter trace segments than a single-frame
 * plan may take), and a frame whose autotuned tiling would raise the LDS of
 * the whole launch above what those rules give is planned by rule.
 */
typedef struct pa_batch pa_batch;

/* Plans a batch (host only: no GPU call, no device pointer dereferenced).
 * frames[i].sensors stay device pointers owned by the caller and must stay
 * valid while the batch is used.  All frames must share ndim.  *out receives
 * a handle to free with pa_batch_destroy. */
pa_status pa_batch_create(const pa_geometry* frames, int32_t n_frames, pa_dtype dtype, pa_batch** out);

/* A batch is planned by the planner's rules.  pa_batch_autotune times the
 * batched A and A^T under those plans and under the frames' recorded tunings
 * (pa_autotune; a tuned frame whose LDS would exceed the rule plans' maximum
 * stays on its rule plan) and keeps the faster set; *tuned (may be NULL) is 1
 * when the tuned plans were kept.  x, y: packed scratch buffers of the batch's
 * sizes (overwritten); workspace: pa_batch_autotune_workspace_bytes() bytes
 * (a candidate needing more than the given size is skipped).  Synchronises
 * the stream.  Query pa_batch_workspace_bytes / pa_batch_cgls_workspace_bytes
 * again afterwards: the plan may have changed. */
size_t pa_batch_autotune_workspace_bytes(const pa_batch* b);
pa_status pa_batch_autotune(pa_batch* b, void* x, void* y, void* workspace, size_t workspace_bytes,
                            void* hip_stream, int32_t* tuned);

/* Frees the handle (and the page-locked host copy of its frame table).  The
 * caller must have synchronised every stream that used it.  NULL is a no-op. */
pa_status pa_batch_destroy(pa_batch* b);

/* x_offsets[i], y_offsets[i] (i = 0..n_frames, either may be NULL): element
 * offset of frame i's image and traces in the packed x and y; entry n_frames
 * is the total. */
pa_status pa_batch_offsets(const pa_batch* b, int64_t* x_offsets, int64_t* y_offsets);

/* Device workspace (bytes, 256-byte aligned, caller-owned) for
 * pa_batch_forward / pa_batch_adjoint, and for pa_batch_cgls_solve with
 * `iters` iterations.  0 means invalid arguments. */
size_t pa_batch_workspace_bytes(const pa_batch* b);
size_t pa_batch_cgls_workspace_bytes(const pa_batch* b, int32_t iters);

/* y := A x and x := A^T y frame by frame (the operators of pa_forward and
 * pa_adjoint).  x, y: packed device buffers of the batch's dtype.  Each call
 * first copies the frame table into the workspace on the stream. */
pa_status pa_batch_forward(pa_batch* b, const void* x, void* y, void* workspace, size_t workspace_bytes,
                           void* hip_stream);
pa_status pa_batch_adjoint(pa_batch* b, const void* y, void* x, void* workspace, size_t workspace_bytes,
                           void* hip_stream);

/* pa_cgls_solve on every frame at once, with one lambda and iteration count
 * and per-frame step sizes and stopping.  history: device double
 * [n_frames][iters + 1][3] in caller frame order, or NULL.  With PA_USE_GRAPH
 * the solve's launches are captured once per argument set and replayed. */
pa_status pa_batch_cgls_solve(pa_batch* b, const void* y, void* x, int32_t iters, double lambda, uint32_t flags,
                              void* workspace, size_t workspace_bytes, double* history, void* hip_stream);

/* After synchronising: stop[i] = iteration at which frame i stopped early, or
 * -1.  Returns PA_ERR_BREAKDOWN when any frame stopped early.  One blocking
 * device-to-host copy. */
pa_status pa_batch_stop_iterations(const pa_batch* b, const void* workspace, int32_t iters, int32_t* stop);

/* ------------------------------------------------------------------ tuning
 * The planner picks the forward operator's tile (base tiles per forward
 * tile) and the adjoint's sensor chunk (from an LDS budget) by rule.
 * pa_autotune times each candidate tiling of both operators on this
 * geometry (best of three runs of eight launches) and records the fastest
 * in a process-wide table keyed by shape (ndim, dtype, nx, ny, nz, S, K and
 * h / (c dt)); every later call on a geometry of that shape, batches
 * included, plans with the recorded tiling.  Tilings change only the order
 * of floating-point sums, not the operator.  x, y: device buffers of the
 * geometry's image and trace sizes, used as scratch (their contents are
 * overwritten).  Synchronises the stream.  Allocates no device memory:
 * the partial-row forward is timed in the caller's workspace. */
typedef struct {
  int32_t fwd_seg;         /* samples of one trace per sensor-major forward work-group (0: no forward work) */
  int32_t adj_lds_bytes;   /* adjoint LDS budget that sets its sensor chunk (0: no adjoint work) */
  int32_t fwd_mode;        /* forward method: 1 = sensor-major, fixed-point tile rows; 2 = sensor-major,
                              FP64 bins; 3 = partial rows (PA_F32 with a workspace; otherwise mode 1);
                              0 under PA_F64, which always uses FP64 bins */
  int32_t fwd_tile[3];     /* mode 3: base tiles per forward tile, per axis */
  double fwd_us, adj_us;   /* measured time per apply of the chosen tilings */
} pa_tuning;

/* Device workspace that lets pa_autotune time the partial-row forward
 * method (PA_F32); 0 when there is nothing to time with it.  Without it (a
 * NULL workspace) pa_autotune times the sensor-major method only. */
size_t pa_autotune_workspace_bytes(const pa_geometry* g, pa_dtype dtype);
pa_status pa_autotune(const pa_geometry* g, pa_dtype dtype, void* x, void* y, void* workspace, size_t workspace_bytes,
                      void* hip_stream, pa_tuning* out);

/* Records t as the tuning of g's shape, as pa_autotune would (for instance
 * one saved from an earlier process).  fwd_us / adj_us are ignored; zero
 * fields keep the planner's rule.  Host only.  PA_ERR_INVALID_ARGUMENT for
 * out-of-range fields, PA_ERR_UNSUPPORTED when the planner cannot take a
 * requested choice (a segment or forward tile whose LDS does not fit, fwd_mode
 * 3 outside PA_F32); nothing is recorded then. */
pa_status pa_tuning_set(const pa_geometry* g, pa_dtype dtype, const pa_tuning* t);

/* Forgets every recorded tiling (later plans use the planner's rules). */
pa_status pa_tuning_clear(void);

/* Message for the last failing call on this thread ("" if none).  Valid until
 * the next pa_* call on the same thread. */
const char* pa_last_error(void);

/* PA_ABI_VERSION of the loaded library. */
int32_t pa_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PA_H */
