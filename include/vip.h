/*
 * vip.h -- C ABI of libvip, an MI355X (gfx950) implementation of the
 * data-parallel hot path of variational full-waveform inversion with SVGD and
 * stochastic SVGD (Zhang & Curtis, "VIP - Variational Inversion Package",
 * arXiv 2310.13325).
 *
 * The inversion layer needs, per particle, the log-posterior value and its
 * gradient (section 3, "Code overview"); the particles are then moved by the
 * SVGD update (eq:phi_mean) or the stochastic SVGD update
 * (eq:stochastic_svgd with the noise of eq:noise_term).  The four calls of
 * that contract are vip_forward, vip_grad_logpost, vip_svgd_step and
 * vip_ssvgd_step; the rest supports them (workspace sizing, tapes for
 * reverse-mode differentiation, batching of several problems, status).
 *
 * Conventions (all calls):
 *  - Units SI (m, s, m/s).  Arrays row-major; a velocity model is [nz][nx]
 *    with x (columns) fastest; a particle ensemble X is [n][d], d = nz*nx,
 *    i.e. the velocity models stacked.
 *  - Pointers marked "device" are HIP device (or managed) memory on the
 *    context's device; "host" pointers are read during the call only.
 *  - Ownership: the caller owns every buffer.  The library never allocates or
 *    frees device memory in a call; scratch comes from a caller workspace
 *    whose size the matching *_workspace query returns.  Workspaces must be
 *    256-byte aligned.
 *  - Execution: work is enqueued asynchronously on the context stream; no call
 *    synchronises except vip_poll and vip_destroy.  Results are bitwise
 *    reproducible for identical inputs (no floating-point atomics).
 *  - Errors: the return value reports host-side validation (shapes, indices,
 *    stability limit, workspace size) and launch failures; nothing is enqueued
 *    when validation fails.  Conditions found on the device (non-finite
 *    values, a velocity above the declared bound, a Cholesky factorisation
 *    that fails after its jitter retries) are latched in a status word inside
 *    the workspace and read with vip_poll.
 *  - One host thread per context.
 */
#ifndef VIP_H
#define VIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VIP_OK = 0,
  VIP_E_ARG = -1,         /* bad shape, null pointer, index outside the grid */
  VIP_E_CFL = -2,         /* vmax*dt*sqrt(4/3 (1/dx^2 + 1/dz^2)) > 1 */
  VIP_E_WORKSPACE = -3,   /* workspace too small or misaligned */
  VIP_E_HIP = -4,         /* HIP runtime error (launch, capture, device) */
  VIP_E_NOT_PD = -5,      /* kernel matrix not positive definite after jitter */
  VIP_E_NONFINITE = -6,   /* NaN / Inf met on the device */
  VIP_E_UNSUPPORTED = -7, /* option not implemented */
  VIP_E_SCRATCH = -8      /* larger than the fixed array of vip_svgd_step_noalloc */
} vip_status;

/* Device status bits latched in a workspace and returned by vip_poll. */
#define VIP_FLAG_NONFINITE   0x1u  /* NaN/Inf in velocity, data, misfit or update */
#define VIP_FLAG_VMAX        0x2u  /* a velocity <= 0 or above vip_grid.vmax */
#define VIP_FLAG_NOT_PD      0x4u  /* Cholesky failed after all jitter retries */
#define VIP_FLAG_JITTER      0x8u  /* Cholesky needed at least one jitter retry */

typedef struct vip_ctx vip_ctx;

/* Finite-difference grid.  The model has nz x nx cells of size dz x dx; the
 * simulation grid adds an absorbing sponge of nb cells on every side
 * (NZ = nz + 2 nb, NX = nx + 2 nb) whose velocity replicates the model's edge
 * cells.  Time samples t_n = n dt, n = 0 .. nt-1.  The scheme is second order
 * in time and fourth order in space for (1/v^2) u_tt - lap u = f, damped by
 * the Cerjan factor g = exp(-(alpha delta_z)^2) exp(-(alpha delta_x)^2),
 * delta = distance into the sponge in cells (the paper's FD method, section
 * 4.2, leaves order and boundary open; these are the readings taken).
 * vmax is an upper bound of every velocity the call may see (e.g. the prior's
 * upper bound); it is checked against the stability limit on the host and
 * against the actual velocities on the device. */
typedef struct {
  int32_t nx, nz, nb, nt;
  double dx, dz, dt;
  double sponge_alpha;
  double vmax;
} vip_grid;

/* Acquisition (section 4.2): ns shots, one point source each, recorded by the
 * same nr receivers.  Indices are interior cell indices (0 <= ix < nx,
 * 0 <= iz < nz), host arrays.  wavelet is the source time function w(t_n),
 * device float [nt]; the source term is w(t_n)/(dx dz) at the shot node
 * (vip_ricker fills a Ricker wavelet).
 * shot_index (host [ns], or NULL for 0 .. ns-1) names the row of the observed
 * data holding each listed shot, and nobs the number of rows (0 .. nobs-1;
 * ignored when shot_index is NULL).  A geometry listing a random subset of a
 * survey's nobs shots, read in place from the full d_obs, gives the minibatch
 * gradients of section 2.4: vip_grad_logpost then scales the misfit of the
 * listed shots by nobs / ns itself (see there). */
typedef struct {
  int32_t ns;
  const int32_t *src_ix, *src_iz;
  int32_t nr;
  const int32_t *rec_ix, *rec_iz;
  const float *wavelet;
  const int32_t *shot_index;
  int32_t nobs;
} vip_geometry;

/* Prior (section 3), per coordinate; all arrays device float [d]:
 *  VIP_PRIOR_NONE.
 *  VIP_PRIOR_UNIFORM_CLIP: uniform on [lo, hi] applied by strategy 1 -- after
 *    an update, values outside the bounds are reset to the nearest bound.  The
 *    log-prior is 0 inside (normalisation dropped), -inf outside; gradient 0.
 *  VIP_PRIOR_UNIFORM_TRANSFORM: uniform on [lo, hi] applied by strategy 2 --
 *    the particles live in the unconstrained space of eq:transform,
 *    theta = log(m - a) - log(b - m), m = a + (b - a) / (1 + exp(-theta)).
 *    vip_grad_logpost then takes theta in vel and returns the log-density of
 *    theta, -J(m) + sum log|dm/dtheta| with dm/dtheta = (m - a)(b - m)/(b - a),
 *    and its gradient with respect to theta, dlogp/dm dm/dtheta
 *    + (a + b - 2m)/(b - a); the SVGD steps do not clip.
 *  VIP_PRIOR_GAUSSIAN: independent normal priors N(mean, std^2): log-prior
 *    -1/2 sum ((m - mean)/std)^2 (constants dropped), gradient
 *    -(m - mean)/std^2; the SVGD steps do not clip.
 * lo, hi are read by the uniform kinds, mean, std by the Gaussian one. */
#define VIP_PRIOR_NONE 0
#define VIP_PRIOR_UNIFORM_CLIP 1
#define VIP_PRIOR_UNIFORM_TRANSFORM 2
#define VIP_PRIOR_GAUSSIAN 3
typedef struct {
  int32_t kind;
  const float *lo, *hi;
  const float *mean, *std;
} vip_prior;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, enqueueing on `stream` (a
 * hipStream_t; NULL = the legacy default stream).  Allocates host-side state
 * and one internal stream used for graph replay; no device memory. */
vip_status vip_create(vip_ctx **ctx, int device, void *stream);
/* Synchronise and release the context (and any cached graphs). */
vip_status vip_destroy(vip_ctx *ctx);
/* Change the stream later calls enqueue on. */
vip_status vip_set_stream(vip_ctx *ctx, void *stream);
/* Graph mode: when on, vip_grad_logpost / vip_forward capture their whole
 * launch sequence into a hipGraph the first time they see a given argument
 * set and replay it afterwards (the arguments, including pointers and the
 * geometry's tables, form the cache key; a context keeps the 32 most recent
 * graphs, evicting the oldest after its replays finish).  Off by default. */
vip_status vip_set_graph_mode(vip_ctx *ctx, int enable);
/* Shape of the time-stepping kernel.  tile = -2 (default) picks a shape per
 * grid; -1 advances one step per launch (each block a 64 x 4*rz tile with its
 * halo staged in LDS); 0 .. vip_tile_count()-1 select a temporally blocked
 * shape that advances up to 4 or 8 steps per launch on an extended tile kept
 * on chip.  Padded grids of 2^29 points or more always use one step per
 * launch (a blocked shape then gives VIP_E_UNSUPPORTED). */
vip_status vip_set_tile(vip_ctx *ctx, int tile);
int vip_tile_count(void);
/* Shape of blocked tile `tile`: shape[0..3] = extended width, extended height
 * (grid points, interior plus a halo of 2 points per step on each side), rows
 * per thread, steps per launch.  VIP_E_ARG for an index out of range. */
vip_status vip_tile_shape(int tile, int32_t shape[4]);
/* 1 if blocked tile `tile` runs persistently (one resident block per compute
 * unit walking a run of tiles, the next tile's state loaded while the current
 * one steps; the same arithmetic, and bitwise the same results, as the
 * non-persistent tile of the same shape), 0 if one block runs per tile,
 * VIP_E_ARG for an index out of range. */
int vip_tile_persistent(int tile);
/* The shape a single-problem call on `grid` over `pairs` (particle, shot)
 * pairs per launch would use with this context's setting: -1 (one step per
 * launch) or a blocked tile index.  pairs <= 0 stands for enough pairs to
 * fill the GPU.  The automatic choice models a launch's time per shape; with
 * fewer blocks than compute units it takes the shape that gives the most. */
vip_status vip_tile_for_grid(const vip_ctx *ctx, const vip_grid *grid, int64_t pairs, int32_t *tile);
/* Human-readable name of a status code (static string). */
const char *vip_status_string(int status);
/* Library version, major*10000 + minor*100 + patch. */
int vip_version(void);

/* Launch timing of the time-stepping kernel.  When enabled (eager mode
 * only), every contiguous run of step-kernel launches of one kind is
 * bracketed by HIP events on the stream it is enqueued on.  vip_read_timing
 * synchronises, sums the runs since the last read per kind (0 = forward,
 * 1 = recompute, 2 = adjoint, 3 = forward that also stores a^n for the
 * adjoint) and forgets them: launches[k], ms[k] (event time of the runs) and
 * point_steps[k] (padded grid points x pairs advanced). */
#define VIP_TIMING_KINDS 4
typedef struct {
  int64_t launches[VIP_TIMING_KINDS];
  double ms[VIP_TIMING_KINDS];
  double point_steps[VIP_TIMING_KINDS];
} vip_timing;
vip_status vip_set_timing(vip_ctx *ctx, int enable);
vip_status vip_read_timing(vip_ctx *ctx, vip_timing *out);

/* Synchronise the context stream, then read and clear the device status word
 * of a workspace previously passed to a call.  *flags gets VIP_FLAG_* bits. */
vip_status vip_poll(vip_ctx *ctx, void *ws, uint32_t *flags);

/* Fill out[n] = (1 - 2 a) exp(-a), a = (pi f0 (n dt - t0))^2, n < nt: the
 * unit-peak Ricker wavelet of section 4.2 (t0 <= 0 selects t0 = 1.5/f0).
 * out: device float [nt]. */
vip_status vip_ricker(vip_ctx *ctx, int32_t nt, double dt, double f0, double t0, float *out);

/* eq:transform for a VIP_PRIOR_UNIFORM_TRANSFORM prior over n particles of d
 * coordinates (device [n][d]): direction 0 maps theta -> m, direction 1 maps
 * m -> theta (m strictly inside (lo, hi); FP64 arithmetic, FP32 out).  in and
 * out may alias.  VIP_E_ARG for another prior kind. */
vip_status vip_prior_transform(vip_ctx *ctx, const vip_prior *prior, int32_t n, int64_t d,
                               const float *in, float *out, int32_t direction);

/* ---- forward modelling ------------------------------------------------- */

/* Workspace bytes for vip_forward with np particles. */
vip_status vip_forward_workspace(const vip_grid *grid, const vip_geometry *geom, int32_t np,
                                 size_t *bytes);

/* Simulate every (particle, shot) pair: data[p][s][n][r] = u_{p,s}^n(x_r),
 * n = 0 .. nt-1 (u^0 = 0), for the velocity models vel (device float
 * [np][nz][nx]).  data: device float [np][ns][nt][nr]. */
vip_status vip_forward(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom, int32_t np,
                       const float *vel, float *data, void *ws, size_t ws_bytes);

/* ---- log-posterior and its gradient ------------------------------------ */

/* Workspace bytes for vip_grad_logpost.  ckpt_every = k: the forward state is
 * stored every k steps and each k-step segment is recomputed once during the
 * adjoint sweep (k >= nt-1 keeps one segment).  stored_steps = S (0 .. nt-1):
 * the last S steps form one segment whose a^n = L u^n + f^n the forward sweep
 * keeps (S slots of a field per live pair), so the adjoint sweep recomputes
 * only the first nt-1-S steps (with the one-step-per-launch kernel the tail
 * is recomputed like any segment).  live_pairs: how many (particle, shot)
 * pairs are simulated at once (0 = all np*ns); memory grows linearly with it.
 * The memory/recompute trade-off changes only FP32 rounding order. */
vip_status vip_grad_logpost_workspace(const vip_grid *grid, const vip_geometry *geom, int32_t np,
                                      int32_t ckpt_every, int32_t stored_steps,
                                      int32_t live_pairs, size_t *bytes);

/* For every particle p (vel[p], device float [np][nz][nx]):
 *   logpost[p] = -J_p + log prior,  J_p = 1/2 sum_{s,n,r} (d_{p,s,n,r} - dobs_{s,n,r})^2 / sigma^2
 * (eq:likelihood with one standard deviation sigma for all samples, constants
 * dropped), and grad[p] = d logpost / d vel[p], obtained by the adjoint-state
 * method (section 3) on the exact discrete adjoint of the forward scheme:
 * forward sweep with checkpoints, then per segment a recompute sweep and an
 * adjoint sweep with the imaging sum accumulated in FP64 (each launch of the
 * step kernel adds its FP32 partial over at most 8 steps) and summed over the
 * shots in FP64.
 * dobs: device float [ns][nt][nr] (or [nobs][nt][nr] read through the
 * geometry's shot_index).  logpost: device double [np].
 * grad: device float [np][nz][nx].  prior may be NULL (no prior).
 * Minibatch (section 2.4, uniformly random data subsets): when the geometry
 * carries a shot_index, its ns listed shots are taken as a subset of the
 * nobs shots of dobs and J is the unbiased estimate
 *   J = (nobs / ns) 1/2 sum_{listed s, n, r} (d - dobs)^2 / sigma^2,
 * whose expectation over uniformly drawn subsets is the full-survey misfit;
 * the residual and the gradient carry the same factor.  sigma is the
 * survey's own noise level (no caller-side scaling). */
vip_status vip_grad_logpost(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom,
                            const vip_prior *prior, int32_t np, const float *vel,
                            const float *dobs, double sigma, int32_t ckpt_every,
                            int32_t stored_steps, int32_t live_pairs, double *logpost,
                            float *grad, void *ws, size_t ws_bytes);

/* Same result through the plain per-pair path: one pair at a time, one launch
 * per time step and per fused-away operation, global-memory stencil.  It exists
 * as the baseline that the batched path is measured against. */
vip_status vip_grad_logpost_plain_workspace(const vip_grid *grid, const vip_geometry *geom,
                                            int32_t np, size_t *bytes);
vip_status vip_grad_logpost_plain(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom,
                                  const vip_prior *prior, int32_t np, const float *vel,
                                  const float *dobs, double sigma, double *logpost, float *grad,
                                  void *ws, size_t ws_bytes);

/* ---- several inversions at once ----------------------------------------- */

/* One inversion problem of a batch: its grid, acquisition, prior, particles,
 * observed data and outputs, with the same meaning as the arguments of
 * vip_grad_logpost. */
typedef struct {
  vip_grid grid;
  vip_geometry geom;
  vip_prior prior;          /* kind VIP_PRIOR_NONE for none */
  int32_t np;
  const float *vel;         /* device [np][nz][nx] */
  const float *dobs;        /* device [ns][nt][nr] */
  double sigma;
  double *logpost;          /* device [np] */
  float *grad;              /* device [np][nz][nx] */
} vip_problem;

#define VIP_MAX_BATCH 4

/* Workspace bytes for vip_grad_logpost_multi (all pairs of all problems live). */
vip_status vip_grad_logpost_multi_workspace(int32_t nprob, const vip_problem *probs,
                                            int32_t ckpt_every, size_t *bytes);

/* vip_grad_logpost for 1 .. VIP_MAX_BATCH independent problems of different
 * grid sizes, shot counts and lengths at once: every launch of the
 * time-stepping kernel carries the next sweep step of every problem that
 * still has one (each block finds its problem, and that problem's sweep mode,
 * from a table in the launch arguments), with one tile shape for the batch
 * (vip_set_tile, or chosen from the batch's estimated cost).  Results equal
 * vip_grad_logpost on each problem alone with the same tile shape, bit for bit. */
vip_status vip_grad_logpost_multi(vip_ctx *ctx, int32_t nprob, const vip_problem *probs,
                                  int32_t ckpt_every, void *ws, size_t ws_bytes);

/* ---- tapes: reverse-mode differentiation of vip_forward ----------------- */

/* Tape bytes: the checkpointed forward states of all np*ns pairs. */
vip_status vip_tape_bytes(const vip_grid *grid, const vip_geometry *geom, int32_t np,
                          int32_t ckpt_every, size_t *bytes);
/* Workspace bytes shared by vip_forward_tape and vip_adjoint_tape. */
vip_status vip_tape_workspace(const vip_grid *grid, const vip_geometry *geom, int32_t np,
                              int32_t ckpt_every, size_t *bytes);
/* vip_forward that also records the checkpoints in `tape` (device). */
vip_status vip_forward_tape(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom,
                            int32_t np, const float *vel, float *data, int32_t ckpt_every,
                            void *tape, size_t tape_bytes, void *ws, size_t ws_bytes);
/* Vector-Jacobian product of vip_forward at vel: grad_vel[p] =
 * sum_{s,n,r} grad_data[p][s][n][r] d data[p][s][n][r] / d vel[p], from the
 * tape written by vip_forward_tape with the same vel and ckpt_every.
 * grad_data: device float [np][ns][nt][nr]; grad_vel: device float
 * [np][nz][nx] (overwritten). */
vip_status vip_adjoint_tape(vip_ctx *ctx, const vip_grid *grid, const vip_geometry *geom,
                            int32_t np, const float *vel, int32_t ckpt_every, const void *tape,
                            size_t tape_bytes, const float *grad_data, float *grad_vel, void *ws,
                            size_t ws_bytes);

/* ---- SVGD / sSVGD ------------------------------------------------------- */

#define VIP_BW_MEDIAN_ALL 0      /* median of all n^2 squared distances (zeros included) */
#define VIP_BW_MEDIAN_OFFDIAG 1  /* median of the n(n-1)/2 distinct pairs */
#define VIP_BW_FIXED 2           /* h = h_fixed */
#define VIP_GRAM_BF16 0          /* X_c X_c^T on BF16 matrix cores, FP32 accumulation */
#define VIP_GRAM_FP32 1          /* X_c X_c^T in FP32 on the FP32 matrix cores */

/* Workspace bytes for vip_svgd_step / vip_ssvgd_step with n particles of
 * dimension d. */
vip_status vip_svgd_workspace(int32_t n, int64_t d, size_t *bytes);

/* Offsets (bytes from the workspace start) of intermediate results that stay
 * valid in the workspace after a step, for inspection:
 * D float [n][n] squared distances, K float [n][n] kernel matrix,
 * h2 double [1] bandwidth h^2, L double [n][n] Cholesky factor of K/n (sSVGD),
 * phi float [n][d] the SVGD direction. */
typedef struct {
  size_t D, K, h2, L, phi;
} vip_svgd_layout;
vip_status vip_svgd_layout_of(int32_t n, int64_t d, vip_svgd_layout *out);

/* One SVGD iteration (eq:rbf, eq:phi_mean) on x (device float [n][d], updated
 * in place) with gradients g = grad log p(x_i) (device float [n][d]):
 *   D_ij = |x_i - x_j|^2;  h^2 = med / (2 ln(n+1)) (h^2 = 1 if med = 0), or h_fixed^2;
 *   K_ij = exp(-D_ij / (2 h^2));  s_i = sum_j K_ij;
 *   phi_i = 1/n [ sum_j K_ij g_j + (s_i x_i - sum_j K_ij x_j) / h^2 ];
 *   x_i <- clip(x_i + eps phi_i) (clip only with a uniform prior).
 * Distances come from the Gram matrix of the centred particles, on BF16 matrix
 * cores or in FP32 (gram_prec).  The product K (G - X_c / h^2) behind phi runs
 * in FP32 on the FP32 matrix cores with VIP_GRAM_FP32; with VIP_GRAM_BF16 it
 * runs on the BF16 matrix cores with K rounded to BF16 and the FP32 operand B
 * = G - X_c / h^2 split into a BF16 pair (B = hi + lo, products K hi + K lo,
 * FP32 accumulation): phi within about 4e-5 relative L2 at n = 2048, a part
 * of the error the BF16 Gram already puts into K.  h2_out: device double [1]
 * or NULL. */
vip_status vip_svgd_step(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g, double eps,
                         int32_t bw_mode, double h_fixed, int32_t gram_prec,
                         const vip_prior *prior, double *h2_out, void *ws, size_t ws_bytes);

/* Step rules for the SVGD update (the optimisers section 2.2 lists for
 * gradient ascent: SGD, AdaGrad, AdaDelta, Adam), applied per coordinate to
 * the direction phi in place of x <- x + eps phi:
 *   SGD       x += eps phi
 *   AdaGrad   s1 += phi^2;                      x += eps phi / (sqrt(s1) + delta)
 *   AdaDelta  s1 = rho s1 + (1 - rho) phi^2;    u = sqrt(s2 + delta) / sqrt(s1 + delta) phi;
 *             s2 = rho s2 + (1 - rho) u^2;      x += eps u          (rho = beta1; eps = 1 is
 *                                                                    the rule as published)
 *   Adam      s1 = b1 s1 + (1 - b1) phi;  s2 = b2 s2 + (1 - b2) phi^2;
 *             x += eps (s1 / (1 - b1^t)) / (sqrt(s2 / (1 - b2^t)) + delta)
 * s1, s2: device float [n][d] state owned by the caller, zero before the first
 * step and carried from step to step (NULL where the rule needs none); t: the
 * 1-based number of this step.  The prior is applied after the step as in
 * vip_svgd_step.  (The sSVGD step keeps its plain form: its noise scale is
 * tied to eps.) */
#define VIP_OPT_SGD 0
#define VIP_OPT_ADAGRAD 1
#define VIP_OPT_ADADELTA 2
#define VIP_OPT_ADAM 3
typedef struct {
  int32_t kind;
  float *s1, *s2;
  int64_t t;
  double beta1, beta2, delta;
} vip_optimizer;
vip_status vip_svgd_step_opt(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g,
                             double eps, int32_t bw_mode, double h_fixed, int32_t gram_prec,
                             const vip_prior *prior, const vip_optimizer *opt, double *h2_out,
                             void *ws, size_t ws_bytes);

/* Kernel of the SVGD / sSVGD steps (section 5): the RBF of eq:rbf, or the
 * diagonal matrix-valued kernel that combines a positive definite diagonal
 * Q with the RBF, Q = inverse per-coordinate variance across the particles
 * (recomputed at every step, ddof 0; q_a = 1 where the variance is 0):
 * K(m, m') = Q^-1 exp(-(m - m')^T Q (m - m') / (2 h^2)).  Its direction is
 *   phi_i = 1/n sum_j k_ij [Q^-1 g_j + (x_i - x_j) / h^2],
 * the median bandwidth taken on the Q-weighted distances, and the sSVGD
 * noise is sqrt(2 eps) L Xi Q^-1/2. */
#define VIP_KERNEL_RBF 0
#define VIP_KERNEL_DIAG_VAR 1

/* One SVGD (noise = 0) or sSVGD (noise = 1) step with every option: bandwidth
 * mode and fixed h, Gram precision, kernel, the sSVGD normals (xi, or Philox
 * seed/stream when xi is NULL) and a step rule (SVGD only; NULL = SGD). */
typedef struct {
  int32_t bw_mode;
  double h_fixed;
  int32_t gram_prec;
  int32_t kernel;
  int32_t noise;
  const float *xi;
  uint64_t seed, stream;
  const vip_optimizer *opt;
} vip_svgd_config;
vip_status vip_svgd_step_ex(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g,
                            double eps, const vip_svgd_config *cfg, const vip_prior *prior,
                            double *h2_out, void *ws, size_t ws_bytes);

/* One stochastic SVGD iteration (eq:stochastic_svgd): the SVGD direction plus
 * noise eta = sqrt(2 eps) L xi per coordinate, L the lower Cholesky factor of
 * K/n (eq:matrixDK, eq:noise_term; factorised in FP64 on the device, with
 * jitter 1e-12 trace/n x10 per retry, at most 6 retries), then the prior clip.
 * n <= 128 factorises in one workgroup with the matrix in LDS; larger n by
 * right-looking 32-column panels over the whole GPU, any n.  A factorisation
 * that needs jitter (numerically coincident particles) reruns in one
 * workgroup with the matrix in global memory: correct, but slow for large n
 * (VIP_FLAG_JITTER reports it).  The direction phi is formed as in
 * vip_svgd_step (with the same Gram precision); the noise product L xi runs
 * over the lower triangle of L on the FP32 matrix cores, or, with the BF16
 * Gram and n > 128, as three BF16 matrix-core products of L and xi each split
 * into a BF16 pair (hi + lo; about 2^-16 relative), and the clip follows it.
 * xi: device float [n][d] standard normals, or NULL to draw them with
 * Philox4x32-10 (key = seed, counter = (element/4, stream)) and Box-Muller. */
vip_status vip_ssvgd_step(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g, double eps,
                          int32_t bw_mode, double h_fixed, int32_t gram_prec,
                          const vip_prior *prior, const float *xi, uint64_t seed, uint64_t stream,
                          double *h2_out, void *ws, size_t ws_bytes);

/* Allocation-free SVGD step, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same step and kernels as vip_svgd_step (same arguments
 * and results), with the workspace replaced by a fixed device array of
 * VIP_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends.  No call allocates or frees memory.
 *  - Size limit: VIP_E_SCRATCH when vip_svgd_workspace(n, d) exceeds
 *    VIP_NOALLOC_SCRATCH_BYTES (e.g. n = 128 at d = 24,000 fits; n = 256 does
 *    not); nothing is enqueued then.
 *  - Sharing: every call on one device uses that device's single array, which
 *    keeps the last call's contents.  Calls that may overlap on one device
 *    (several streams, threads or contexts) race on it: serialise them.
 *  - status: device uint32 that the step ORs its VIP_FLAG_* bits into (the
 *    caller clears it), or NULL to drop them. */
#define VIP_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
vip_status vip_svgd_step_noalloc(vip_ctx *ctx, int32_t n, int64_t d, float *x, const float *g,
                                 double eps, int32_t bw_mode, double h_fixed, int32_t gram_prec,
                                 const vip_prior *prior, double *h2_out, uint32_t *status);

/* Several independent ensembles, each updated as by vip_svgd_step or
 * vip_ssvgd_step (ensemble e draws its Philox normals from stream + e when its
 * xi is NULL); the workspace is shared (vip_svgd_multi_workspace) and the
 * status word of its first bytes collects every ensemble's flags. */
typedef struct {
  int32_t n;
  int64_t d;
  float *x;                 /* device [n][d], updated in place */
  const float *g;           /* device [n][d] */
  double eps;
  vip_prior prior;
  const float *xi;          /* device [n][d] or NULL (sSVGD only) */
  double *h2_out;           /* device [1] or NULL */
} vip_ensemble;
vip_status vip_svgd_multi_workspace(int32_t nens, const vip_ensemble *ens, size_t *bytes);
vip_status vip_svgd_step_multi(vip_ctx *ctx, int32_t nens, const vip_ensemble *ens, int32_t bw_mode,
                               double h_fixed, int32_t gram_prec, void *ws, size_t ws_bytes);
vip_status vip_ssvgd_step_multi(vip_ctx *ctx, int32_t nens, const vip_ensemble *ens,
                                int32_t bw_mode, double h_fixed, int32_t gram_prec, uint64_t seed,
                                uint64_t stream, void *ws, size_t ws_bytes);

/* Automatic differentiation variational inference (section 2.2: eq:normal,
 * eq:argmaxELBO_advi, eq:gradient_mu, eq:gradient_L; the mean-field family of
 * section 5).  The variational family is q(theta) = N(mu, L L^T) in the
 * unconstrained space theta = T(m) of eq:transform; the per-sample gradients
 * g_s = grad_theta log p(theta_s, d) that the step consumes are what
 * vip_grad_logpost returns for the samples theta_s under the
 * VIP_PRIOR_UNIFORM_TRANSFORM prior (or the Gaussian prior, T = identity;
 * the clip prior has no place in ADVI).  An iteration is: draw eta
 * (vip_philox_normals), vip_advi_sample, vip_grad_logpost on the S samples,
 * vip_advi_step.
 *  family VIP_ADVI_FULL_RANK: L is device float [d][ldl], row-major, ldl >= d,
 *    lower triangular; only entries j <= i are read or written (the rest of
 *    the array is never touched).
 *  family VIP_ADVI_MEAN_FIELD: L is device float [d], the diagonal of a
 *    diagonal L (ldl is ignored).
 * mu: device float [d].  eta, theta, g: device float [S][d], S the number of
 * Monte Carlo samples, 1 <= S <= VIP_ADVI_MAX_SAMPLES.  No call allocates or
 * synchronises; VIP_E_ARG for a bad family, size or pointer. */
#define VIP_ADVI_FULL_RANK 0
#define VIP_ADVI_MEAN_FIELD 1
#define VIP_ADVI_MAX_SAMPLES 32

/* theta[s] = mu + L eta[s] for every sample s (FP32 arithmetic; the full-rank
 * product sums in a fixed order, so results are reproducible). */
vip_status vip_advi_sample(vip_ctx *ctx, int32_t family, int64_t d, int32_t S, const float *mu,
                           const float *L, int64_t ldl, const float *eta, float *theta);

/* One ascent step of the ELBO from the samples of vip_advi_sample (same mu, L,
 * eta) and their gradients g:
 *   grad_mu = 1/S sum_s g[s]                                  (eq:gradient_mu)
 *   grad_L  = 1/S sum_s g[s] eta[s]^T + (L^-1)^T              (eq:gradient_L)
 * on the free entries (the lower triangle, or the diagonal for the mean
 * field; the lower part of (L^-1)^T is diag(1 / L_ii)), then
 *   mu += rule(grad_mu),  L += rule(grad_L)
 * with the step rules of vip_svgd_step_opt (eps and the rule's formula as
 * there; NULL = SGD).  opt_mu's state arrays are device float [d]; opt_L's
 * have L's layout ([d][ldl] with the same ldl, or [d]); each is zero before
 * the first step.  The diagonal of L must be nonzero.
 * grad_mu ([d]) and grad_L (L's layout, lower entries only): device float
 * outputs of the two gradients, or NULL.
 * elbo: device double [1] or NULL; when given, logpost (device double [S],
 * the samples' log p(theta_s, d) from vip_grad_logpost) is required and
 *   elbo = 1/S sum_s logpost[s] + sum_i log|L_ii| + d/2 (1 + log 2 pi)
 * is written from L before the step (eq:argmaxELBO_advi, up to the constant
 * the log-posterior drops). */
vip_status vip_advi_step(vip_ctx *ctx, int32_t family, int64_t d, int32_t S, float *mu, float *L,
                         int64_t ldl, const float *eta, const float *g, double eps,
                         const vip_optimizer *opt_mu, const vip_optimizer *opt_L, float *grad_mu,
                         float *grad_L, const double *logpost, double *elbo);

/* Standard normals out[e], e < count, from Philox4x32-10 as described for
 * vip_ssvgd_step (device float [count]). */
vip_status vip_philox_normals(vip_ctx *ctx, int64_t count, uint64_t seed, uint64_t stream,
                              float *out);
/* The raw Philox4x32-10 words behind vip_philox_normals: out[4q + w] = word w
 * of the block with counter (q, stream) and key seed, q < nblocks
 * (device uint32 [4 nblocks]). */
vip_status vip_philox_uint32(vip_ctx *ctx, int64_t nblocks, uint64_t seed, uint64_t stream,
                             uint32_t *out);

#ifdef __cplusplus
}
#endif

#endif /* VIP_H */
