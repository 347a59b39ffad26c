/*
 * eswave.h -- C ABI of the MI355X (gfx950) wavelet Sobolev-embedding / Matern-prior library.
 *
 * Paper: Kultima, Ramlau, Sahlstrom, Tarvainen, "Fast reconstruction approaches for
 * photoacoustic tomography with smoothing Sobolev/Matern priors", arXiv 2507.02401.
 *
 * The library applies, on the GPU and in FP32, the wavelet realisation of the adjoint
 * Sobolev embedding of Sec. 4 (Prop. 4.2, the per-level weight rule and the block
 * diagonal D, and the closing formula E_s^* X = W^{-1}(D (W X))):
 *
 *   W      periodic orthonormal Daubechies (dbN, L = 2N taps, extremal phase) DWT of depth m,
 *          separable over 1, 2 or 3 axes (Mallat's isotropic pyramid, Sec. 4 / Def. 4.1);
 *   D_tau  diagonal, weight 1 on the approximation band and 2^{-tau s (m-i)} on every detail
 *          band of level i (1 = finest, m = coarsest).
 *
 *   es_adjoint(x)        = D_s W x           E_s^* in orthonormal coordinates of H^s
 *   es_apply(c)          = W^T D_s c         E_s, its Euclidean adjoint
 *   matern_cov_apply(x)  = W^T D_{2s} W x    = E_s E_s^*: the paper's pixel-space E_s^*; with
 *                                            s = nu + d/2 the Matern covariance of Prop. 3.2
 *                                            up to its constant (dropped, Remark 3.3)
 *   matern_sample(xi)    = W^T D_s W xi      symmetric square root of the covariance; applied to
 *                                            white noise it draws a prior sample (Sec. 3, the
 *                                            Gaussian prior of the MAP estimate)
 *
 * Data layout.  Every array is FP32, contiguous, row-major (last axis fastest).  A call
 * processes `batch` independent instances of the same geometry stored back to back
 * (instance b starts at element b * prod(shape)).  Coefficient arrays use the packed
 * pyramid layout: same shape as the image; after m levels the approximation occupies
 * [0, n_k/2^m) on every axis k and the detail band of level i with high-pass pattern
 * eps in {0,1}^d \ {0} occupies [eps_k n_k/2^i, (eps_k+1) n_k/2^i) on axis k.
 * The 1-D step is the periodic correlation a[k] = sum_t h[t] x[(2k+t) mod n],
 * d[k] = sum_t g[t] x[(2k+t) mod n], g[t] = (-1)^t h[L-1-t].
 *
 * Arguments shared by the operator entry points:
 *   ndim     1, 2 or 3.
 *   shape    host array of ndim sides; every side must be divisible by 2^levels and
 *            at least 2^levels (non-square grids allowed).
 *   batch    number of instances (>= 0; 0 is a no-op).
 *   order    Daubechies order N in 1..8 (1 = Haar).
 *   levels   depth m >= 0 (0 gives the identity); at most 30.
 *   s        smoothness, finite, any sign (s < 0 gives the inverse operators' weights).
 *   in/out   device pointers, 16-byte aligned, batch*prod(shape) floats each, caller-owned,
 *            must not overlap.
 *   ws       device workspace of at least es_workspace_bytes(...) bytes, 256-byte aligned
 *            (may be NULL when that size is 0); caller-owned, contents undefined on return.
 *   stream   hipStream_t to launch on (NULL = default stream).  Launches are asynchronous.
 *
 * Errors.  Every entry point returns an es_status, never throws and never aborts.  All
 * arguments are validated on the host before any device call; on a non-OK status no
 * work was enqueued (except ES_EDEVICE, reported by the HIP runtime at launch).
 * es_last_error() returns a thread-local message for the last non-OK status.
 * Thread safety: entry points may be called concurrently from several threads.
 */
#ifndef ESWAVE_H
#define ESWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ES_OK = 0,
  ES_EINVAL = 1,       /* bad argument: ndim, shape, order, levels, s, pointer, overlap, alignment */
  ES_EWORKSPACE = 2,   /* workspace missing or smaller than es_workspace_bytes()                     */
  ES_EUNSUPPORTED = 3, /* valid request this build cannot run (e.g. no gfx950 device)               */
  ES_EDEVICE = 4,      /* HIP runtime error; message from hipGetErrorString in es_last_error()      */
  ES_ENOMEM = 5        /* host or device allocation failed (plans, FFT plans, GMRES host state)     */
} es_status;

typedef enum { ES_OP_ADJOINT = 0, ES_OP_APPLY = 1, ES_OP_COV = 2, ES_OP_SAMPLE = 3 } es_op;

/* ---- single-geometry entry points (uniform batch) ------------------------------------- */

/* E_s^* in wavelet coordinates: coeff = D_s W x (Sec. 4, Prop. 4.2 and the weight rule). */
es_status es_adjoint(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                     const float* x, float* coeff, void* ws, size_t ws_bytes, void* stream);

/* E_s = (E_s^*)^T: x = W^T D_s coeff (exact transpose of es_adjoint). */
es_status es_apply(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                   const float* coeff, float* x, void* ws, size_t ws_bytes, void* stream);

/* y = W^T D_{2s} W x: the paper's pixel-space E_s^* (Sec. 4, closing formula). */
es_status matern_cov_apply(int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                           double s, const float* x, float* y, void* ws, size_t ws_bytes, void* stream);

/* x = W^T D_s W xi: symmetric square root of matern_cov_apply (prior sampling). */
es_status matern_sample(int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                        double s, const float* xi, float* x, void* ws, size_t ws_bytes, void* stream);

/* Allocation-free variant of matern_cov_apply, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
 * operator, kernels and results, with the workspace taken from a fixed scratch array the library
 * holds on each device (es_noalloc_scratch_bytes() bytes, 64 MiB, allocated with the library's code
 * object on that device and kept until the process ends).  Calls no hipMalloc/hipFree and
 * allocates no device memory.  The caller passes x and y as for matern_cov_apply.
 * Errors: ES_EWORKSPACE when es_workspace_bytes(ndim, shape, batch, order, levels, ES_OP_COV)
 * exceeds the scratch size (no work is enqueued); otherwise as matern_cov_apply.
 * All calls on one device share that device's scratch and leave their level arrays in it: calls
 * that overlap in time on one device (two streams, two threads) race and give undefined results;
 * calls ordered on one stream do not. */
es_status matern_cov_apply_noalloc(int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                                   double s, const float* x, float* y, void* stream);
size_t es_noalloc_scratch_bytes(void);

/* Workspace bytes the four entry points above need for this geometry and op (es_op). */
size_t es_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels, int op);

/* Reference variant of the four operators: one launch per 1-D pass per level per instance
 * (no fusion across axes or levels), for comparison against the fused path.  Same
 * arguments and results; needs es_workspace_bytes_plain(...) bytes of workspace. */
es_status es_plain_apply_op(int op, int ndim, const int64_t* shape, int64_t batch, int order,
                            int levels, double s, const float* in, float* out, void* ws,
                            size_t ws_bytes, void* stream);
size_t es_workspace_bytes_plain(int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                                int op);

/* ---- squared H^s norm ------------------------------------------------------------------- */

/* norms[b] = ||x_b||^2_{H^s} = ||D_{-s} W x_b||^2 = sum over the orthonormal coefficients c = W x_b
 * of 2^{2 s j} c^2 (detail level i: j = m - i; approximation: weight 1), the squared norm that
 * defines the prior (Sec. 3, ||x||_{H^s} = ||Gamma x||, with the wavelet weights of Sec. 4).  Its
 * gradient is 2 W^T D_{-2s} W x = 2 * matern_cov_apply(x) with smoothness -s.  The analysis runs
 * in squared-norm mode (coefficients are squared and summed per work-group, never stored).  All
 * sums are FP32 with compensation (Neumaier per thread, error-free pair sums across threads and
 * work-groups) in a fixed order, so results are deterministic and, the terms being non-negative,
 * within a few FP32 roundings of the exact sum of the computed squares.
 * x: device, batch * prod(shape) floats, 16-byte aligned.  norms: device, batch floats, 4-byte
 * aligned.  ws: device, es_hs_norm_workspace_bytes(...) bytes, 256-byte aligned.  Other
 * arguments and errors as for es_adjoint. */
es_status es_hs_norm_sq(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                        const float* x, float* norms, void* ws, size_t ws_bytes, void* stream);
size_t es_hs_norm_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels);

/* ---- matrix-free Tikhonov / MAP solver around the prior ----------------------------------- */

/* Solves, per instance, the normal equations of J(x) = 1/2 ||M x - p||^2 + alpha/2 ||x||^2_{H^s}
 * (Sec. 3: the Tikhonov functional and the linear equation of its minimiser; Sec. 4: iterative
 * solvers such as conjugate gradients on the wavelet form):
 *     (M + alpha W^T D_{-2s} W) x = M p,   M = diag(mask),
 * by conjugate gradients preconditioned with W^T D_{2s} W = matern_cov_apply(s), starting from
 * x = 0.  Every step runs on the device: two operator applications per iteration (matern_cov_apply
 * with -s and +s) and fused element-wise update / inner-product kernels; inner products are FP32
 * with compensated per-thread sums, pairwise trees and a fixed-order per-instance reduction
 * (deterministic).  An instance stops changing once ||r|| / ||M p|| <= rtol; the host reads the
 * residuals every `check_every` iterations (synchronising `stream`) and stops when all instances
 * are below rtol or after max_iter iterations.
 *   p, mask, x   device, batch * prod(shape) floats, 16-byte aligned; x is written (must not
 *                overlap p, mask or ws).
 *   iterations   host, receives the iterations run (may be NULL).
 *   rel_residual host, batch floats: ||r|| / ||M p|| of each instance at the end (0 when M p = 0).
 *   ws           device, es_tikhonov_pcg_workspace_bytes(...) bytes, 256-byte aligned: r, z, d, A d,
 *                partial sums, per-instance scalars and the operator's workspace.
 * Other arguments as for matern_cov_apply.  Errors: ES_EINVAL (arguments, alpha <= 0, rtol < 0,
 * max_iter < 0), ES_EWORKSPACE, ES_EUNSUPPORTED, ES_EDEVICE.  Synchronous on return. */
es_status es_tikhonov_pcg(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                          double alpha, const float* p, const float* mask, float* x, int32_t max_iter, double rtol,
                          int32_t check_every, int32_t* iterations, float* rel_residual, void* ws, size_t ws_bytes,
                          void* stream);
size_t es_tikhonov_pcg_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels);

/* Solves, per instance, the regularised linear system in the form the paper writes it (Sec. 3:
 * the linear equation of the Tikhonov minimiser, E_s^* applied to its normal equations; Sec. 5:
 * solved there by GMRES):
 *     (E_s^* K^* K + alpha I) x = E_s^* K^* p,   K = diag(mask),  E_s^* = W^T D_{2s} W,
 * by restarted GMRES from x = 0.  E_s^* is matern_cov_apply(s); the system is not symmetric.  For a
 * 0/1 mask its solution is that of es_tikhonov_pcg.  Arnoldi step: one operator application, then
 * classical Gram-Schmidt with one reorthogonalisation pass, the second pass written through the
 * basis's Gram matrix: one pass of inner products over the basis (with the new vector and with the
 * newest basis vector), coefficients c = 2h - G h, one update pass; all on the device (FP32
 * vectors, compensated FP32 inner products reduced per instance in a fixed order: deterministic).  The host
 * reads the new Hessenberg column after every step (synchronising `stream`) and keeps the
 * Hessenberg matrix, its Givens rotations and the least-squares solution in FP64.  An instance
 * stops contributing once its residual estimate |g_{k+1}| / ||E_s^* K^* p|| <= rtol; after every
 * `restart` steps the iterate is formed (x += V y) and, if any instance is still above rtol and
 * iterations remain, GMRES restarts from the true residual.  At most max_iter Arnoldi steps.
 *   restart      basis length, 1..64.
 *   p, mask, x   device, batch * prod(shape) floats, 16-byte aligned; x is written (must not
 *                overlap p, mask or ws).
 *   iterations   host, receives the Arnoldi steps run (may be NULL).
 *   rel_residual host, batch floats: the true ||E_s^* K^* p - A x|| / ||E_s^* K^* p|| of each
 *                instance at the end (one more operator application; 0 when the right side is 0).
 *   ws           device, es_tikhonov_gmres_workspace_bytes(...) bytes, 256-byte aligned: the basis
 *                (restart + 1 vectors), the right side, two work vectors, partial sums, the
 *                per-instance coefficients and the operator's workspace.
 * Other arguments as for matern_cov_apply.  Errors: ES_EINVAL (arguments, alpha <= 0, rtol < 0,
 * max_iter < 0, restart outside 1..64), ES_EWORKSPACE, ES_ENOMEM (host memory for the per-instance
 * least-squares state), ES_EUNSUPPORTED, ES_EDEVICE.  Synchronous on
 * return. */
es_status es_tikhonov_gmres(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                            double alpha, const float* p, const float* mask, float* x, int32_t restart,
                            int32_t max_iter, double rtol, int32_t* iterations, float* rel_residual, void* ws,
                            size_t ws_bytes, void* stream);
size_t es_tikhonov_gmres_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                                         int32_t restart);

/* ---- Fourier form of E_s^* (Sec. 4, Implementation) ------------------------------------ */

/* y_b = ifft(B . fft(x_b)) for each of `batch` instances: the paper's second realisation of the
 * adjoint embedding, multiplication of the spectrum by the Bessel potential
 * B[k] = (1 + 4 pi^2 sum_a (k_a / period)^2)^(-s) (proof of Prop. 3.2; Sec. 4, Implementation), where the grid samples
 * a periodic box of side `period` on every axis and k_a in -n_a/2 .. n_a/2 - 1 is the integer
 * frequency of axis a.  It is a different operator from matern_cov_apply (diagonal in the Fourier
 * basis, shift-invariant; the two are norm-equivalent on the detail scales), with the same role.
 * The transforms are hipFFT's (real-to-complex and complex-to-real); the multiplication by B and
 * the 1/N of the inverse transform are one pass of this library over the half spectrum.
 *   ndim, shape  1..3 axes, every side in 2..2^30 (any length, not only powers of two); at most
 *                2^31-1 elements per instance.
 *   s            finite, any sign (s < 0 multiplies by the inverse potential; |s| must keep
 *                B within FP32 range).  period: finite, > 0 (1 = unit box).
 *   x, y         device, batch * prod(shape) floats, 16-byte aligned.  y == x (in place) is
 *                allowed; other overlaps are not.  When y != x, x is copied into y first (the
 *                FFT library may overwrite the input of an out-of-place transform): x is never
 *                written.
 *   ws           device workspace of es_fft_workspace_bytes(...) bytes, 256-byte aligned, not
 *                overlapping x or y: the half spectrum (batch * prod(shape[:-1]) * (n_last/2+1)
 *                complex FP32) followed by hipFFT's work area.
 * The first call for a geometry and batch (or its workspace query) creates a pair of hipFFT plans
 * on the current device and caches them; plan creation allocates the library's own device tables,
 * held until es_fft_release_plans().  Calls are serialised by a lock (plans hold their stream and
 * work area), so concurrent calls from several threads are safe but do not overlap on the host.
 * Errors: ES_EINVAL, ES_EWORKSPACE, ES_EUNSUPPORTED (not gfx950), ES_ENOMEM (plan allocation),
 * ES_EDEVICE (HIP or hipFFT error, named in es_last_error()). */
es_status es_fft_cov_apply(int ndim, const int64_t* shape, int64_t batch, double s, double period, const float* x,
                           float* y, void* ws, size_t ws_bytes, void* stream);
/* Workspace bytes of es_fft_cov_apply for this geometry and batch (creates the plans if needed). */
es_status es_fft_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, size_t* bytes);
/* Waits for every device that holds cached plans and destroys them. */
es_status es_fft_release_plans(void);

/* ---- non-periodic transform (Sec. 4, the fast wavelet transform with band lengths l(i)) ---- */

/* y_b = W^{-1} D_{2s} W x_b with W the non-periodic DWT of depth `levels` that Sec. 4 evaluates
 * with MATLAB's fast wavelet transform: half-point symmetric extension (the signal mirrored about
 * its ends, end samples repeated), one step of a length-n axis keeping
 *     a[k] = sum_t h[t] x_ext[2k + t - (L-2)],  d[k] = sum_t g[t] x_ext[2k + t - (L-2)],
 *     k < l = floor((n + L - 1) / 2)   (the book-keeping lengths, es_sym_band_lengths),
 * separable over the axes of the approximation block, and W^{-1} its left inverse (keeps the
 * central n samples of the upsampled, filtered bands; not W^T: the transform is redundant and not
 * orthogonal, so the operator is not symmetric).  D weights detail level i by 2^{-2s(m-i)} and the
 * approximation by 1, as for matern_cov_apply.  Only the all-low band of each level is formed (the
 * projection form, exact because the synthesis halves S_a, S_d satisfy S_a A + S_d B = I).
 *   ndim, shape  1..3 axes, every side in 1..2^30 (any length; no divisibility condition); every
 *                level at most 2^31-1 elements per instance (levels may grow for sides < L - 1).
 *   order 1..8, levels 0..30 (levels <= 1 give the identity), s finite, any sign.
 *   x, y         device, batch * prod(shape) floats, 16-byte aligned, must not overlap.
 *   ws           device, es_sym_workspace_bytes(...) bytes (the arrays a_1 .. a_{m-1}), 256-byte
 *                aligned, may be NULL when that size is 0.
 * Errors: ES_EINVAL (arguments, overlap, alignment), ES_EWORKSPACE, ES_EUNSUPPORTED, ES_EDEVICE;
 * all checks on the host before any launch.  Asynchronous on `stream`. */
es_status es_sym_cov_apply(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                           const float* x, float* y, void* ws, size_t ws_bytes, void* stream);
/* Workspace bytes of es_sym_cov_apply (0 for invalid arguments or batch <= 0). */
size_t es_sym_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels);
/* x_b = (W^{-1} D_{2s} W)^T y_b = W^T D_{2s} W^{-T} y_b: the transpose of es_sym_cov_apply (the
 * operator is not symmetric), for gradients of losses through it.  Evaluated as
 * w_1 y + sum_i c_i (A^T)^i (S_a^T)^i y with S_a^T the analysis sum over the signal extended by
 * zeros and A^T the synthesis onto the extension positions -(L-2) .. 2l-1 folded back onto the
 * samples they reflect to.  Arguments as for es_sym_cov_apply (y in, x out); the workspace is
 * es_sym_transpose_workspace_bytes(...) bytes (the level arrays; on 3-D grids also one extended
 * level, since 1-D and 2-D grids fold the extension in a pass over the boundary shell only). */
es_status es_sym_cov_apply_transpose(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                                     const float* y, float* x, void* ws, size_t ws_bytes, void* stream);
size_t es_sym_transpose_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels);
/* Band lengths l_1 .. l_levels of one axis of length n (host array of `levels` entries). */
es_status es_sym_band_lengths(int64_t n, int order, int levels, int64_t* lengths);

/* ---- ragged batches: many geometries in one captured launch sequence ------------------ */

typedef struct {
  int32_t ndim;
  int32_t order;
  int64_t shape[3];
  int32_t levels;
  int32_t reserved;
  double s;
} es_desc;

typedef struct es_plan es_plan;

/* Builds a plan for `count` instances (descs is a host array) of one op.  The plan owns its
 * device descriptor tables and a hipGraph of the whole launch sequence; the graph is
 * instantiated on the first es_plan_execute.  Returns ES_ENOMEM if allocation fails.
 *
 * By default a plan runs phase-merged launches: one launch per level phase and kernel, every
 * instance of the phase in it.  With the environment variable ESWAVE_PLAN_PERSISTENT=1 at
 * creation, plans of matern_cov_apply / matern_sample run persistently instead: one kernel
 * launch per (dimensionality, filter length) present in the plan, the launches running
 * concurrently as branches of the plan's graph, runs every level tile and coarse block of every
 * instance (identity instances: copies), each work-group
 * taking the next work item from a queue in device memory and waiting, with a bounded poll, until
 * the previous step of the same instance has finished.  The item order interleaves instances so
 * that coarse levels of one overlap fine levels of others; its pipeline lag and the largest block
 * the coarse step takes in LDS (coarse fusion depth) are chosen by es_plan_autotune.  Plans whose
 * level arrays cannot take the vector staging path, and plans of es_adjoint / es_apply, run
 * phase-merged.  Persistent plans use twice the workspace (every level array written once). */
es_status es_plan_create(const es_desc* descs, int32_t count, int op, void* stream, es_plan** out);

/* Runs the plan: in[i] / out[i] (host arrays of device pointers) are instance i's input and
 * output.  When the pointers equal those of the previous call the captured graph is
 * replayed as is; otherwise the descriptor table is refreshed first. */
es_status es_plan_execute(es_plan* plan, const float* const* in, float* const* out, void* ws,
                          size_t ws_bytes, void* stream);

/* Same as es_plan_execute but launches kernel by kernel without the graph (for comparison). */
es_status es_plan_execute_eager(es_plan* plan, const float* const* in, float* const* out, void* ws,
                                size_t ws_bytes, void* stream);

size_t es_plan_workspace_bytes(const es_plan* plan);
/* Number of kernel launches one execution of the plan performs. */
int32_t es_plan_num_launches(const es_plan* plan);
void es_plan_destroy(es_plan* plan);

/* 1 when the plan runs persistently (see es_plan_create), else 0. */
int32_t es_plan_is_persistent(const es_plan* plan);

/* After an execution: synchronises `stream` and reads the persistent launches' error words.
 * ES_EDEVICE when a dependency wait gave up after its poll limit (the results of that execution
 * are invalid; the kernels still ran to completion); ES_OK otherwise, and for plans that do not
 * run persistently. */
es_status es_plan_errors(es_plan* plan, void* stream);

/* Tunes the plan on the caller's buffers by timing candidates (eager launches, HIP events on
 * `stream`, synchronising; fastest of three rounds of `reps` executions), keeps the fastest and
 * leaves the tuned plan's result in `out`; the captured graph is rebuilt on the next
 * es_plan_execute.
 *   Phase-merged plans: (1) for matern_cov_apply / matern_sample, the coarse fusion depth (largest
 *   block the coarse-level kernel takes: 16384, 4096 or 1024 floats), each candidate a plan rebuilt
 *   with that limit and timed as a whole; (2) the tile choice of every merged launch (tile variant,
 *   and kernel family where a level has two), launches with the most work-groups first, each
 *   candidate timed inside the whole plan.
 *   Persistent plans: the coarse fusion depth (2048 or 512 floats) and the pipeline lag of the item
 *   order.
 * Tile choices give identical results; the coarse fusion depth changes the summation order, so
 * results of different depths agree to rounding only.  Same pointer rules as es_plan_execute. */
es_status es_plan_autotune(es_plan* plan, const float* const* in, float* const* out, void* ws, size_t ws_bytes,
                           int32_t reps, void* stream);

/* The configuration in use: coarse limit (floats; -1 for a phase-merged plan on the default limit),
 * pipeline lag and work items per execution (-1.0 and 0 for plans that do not run persistently). */
es_status es_plan_config(const es_plan* plan, int64_t* coarse_limit, double* lag, int64_t* items);

/* Host-only plan checks (instrumentation; no device call, usable without a GPU).
 * A plan freezes every instance's launch sequence (kernels, tile variants, tile counts, vector
 * path, coarse-kernel LDS class) at creation; executions only move the frozen launches' pointers
 * onto the caller's buffers, and every launch's memory footprint (the block each array is
 * addressed with, per instance) is checked against those buffers before anything is enqueued.
 * es_plan_create_host builds the same host-side plan as es_plan_create without device
 * resources (such a plan cannot be executed; destroy it with es_plan_destroy).
 * es_plan_fill_host runs the checks and table fill of an execution for the given addresses
 * (plain integers, never dereferenced): in[i] / out[i] of instance i, ws of ws_bytes bytes.
 * Returns ES_OK, or ES_EINVAL / ES_EWORKSPACE with the offending instance and step in
 * es_last_error().  es_plan_work_groups: work-groups (phase-merged plans) or work items
 * (persistent plans) of one execution, after a fill. */
es_status es_plan_create_host(const es_desc* descs, int32_t count, int op, es_plan** out);
es_status es_plan_fill_host(es_plan* plan, const uint64_t* in, const uint64_t* out, uint64_t ws, size_t ws_bytes);
int64_t es_plan_work_groups(const es_plan* plan);

/* ---- autotuning ------------------------------------------------------------------------- */

/* Chooses, for every launch of the operator's launch sequence for this geometry and batch, among
 * its candidates -- the tile variants, and for levels with two kernel families (plain tiles /
 * tiles streamed along the slowest axis) the variants of both.  Each candidate is timed inside
 * the whole sequence (HIP events on `stream`, synchronising; three round-robin rounds of `reps`
 * sequences, fastest round kept), launch by launch in sequence order.  The choices go to a
 * process-wide cache used by later calls with the same geometry, and the correct result of the
 * operator is left in `out`.  Arguments as for the operator entry
 * points.  With the environment variable ESWAVE_TUNE_CACHE naming a file, choices are appended
 * there and read back by later processes.  Candidates change only the speed: results are
 * bit-identical. */
es_status es_autotune(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                      double s, const float* in, float* out, void* ws, size_t ws_bytes, int32_t reps,
                      void* stream);

/* ---- instrumentation: the launch sequence of one operator call ------------------------- */

/* Number of kernel launches es_adjoint / es_apply / matern_cov_apply / matern_sample (op) run
 * for this geometry (0 when the operator is the identity, -1 on invalid arguments). */
int32_t es_schedule_length(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels);

/* Names launch `index` of that sequence (kernel kind, dimensionality, taps, tile variant),
 * its work-group count and the pyramid level it works on.  Host only. */
es_status es_schedule_describe(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                               int32_t index, char* name, size_t name_len, int64_t* work_groups, int32_t* level);

/* Enqueues only launch `index` of the sequence, with the same arguments as the operator call;
 * the launches before it must already have run on the same buffers.  Used to time one kernel. */
es_status es_schedule_run_step(int op, int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                               double s, const float* in, float* out, void* ws, size_t ws_bytes, int32_t index,
                               void* stream);

/* ---- host-side helpers (no device call) ------------------------------------------------ */

/* Daubechies extremal-phase low-pass filter dbN (2*order doubles) as this library derives
 * it on the host; the kernels use it rounded to FP32.  ES_EINVAL for order outside 1..8. */
es_status es_filter(int order, double* h_out);

/* Weight of the detail bands of each level i = 1..levels (index i-1) and of the
 * approximation (index levels), as FP32 values the kernels use; tau = 2 for the covariance,
 * 1 for es_adjoint / es_apply / the sampler. */
es_status es_level_weights(int levels, double s, double tau, float* w_out);

const char* es_status_string(es_status status);
const char* es_last_error(void);
const char* es_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ESWAVE_H */
