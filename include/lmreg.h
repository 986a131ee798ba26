/*
 * lmreg — one factored Levenberg–Marquardt (LM) step of dense 3D image
 * registration on AMD Instinct MI355X (gfx950).
 *
 * Method: "Factored Levenberg–Marquardt for Diffeomorphic Image
 * Registration" (arXiv 2603.19371).  One LM attempt on a pair (F, M) with
 * displacement field u:
 *   1. closed-form damped rank-1 step  du = -r g / (|g|^2 + lambda)
 *      (Sec. 2.2, eq. tile1; derivation in App. A), with g the smoothed
 *      gradient of the accepted field and r = 1 - LNCC its residual
 *      (Sec. 2.2, squared-loss form of LNCC);
 *   2. compositive integration  u~ = eps du + u o (Id + eps du)
 *      (Sec. 2.1, eq. compositive);
 *   3. loss of the candidate  L = -mean_x cc(x), cc the windowed squared
 *      correlation of F and M o (Id + u~) (Sec. 1, eq. 1; Sec. 2.2);
 *   4. damping rule (Sec. 2.2, eq. lambda-update) and rejection test
 *      (Sec. 2.2, eq. delta-loss; Sec. 3.4, eq. rejection), decided on the
 *      device from an FP64 reduction of the loss;
 *   5. if accepted, the analytic gradient of the loss with respect to u,
 *      Gaussian-smoothed (Eulerian descent, Sec. 2.1), for the next attempt.
 *
 * Conventions for every call:
 *   - Volumes are dense [nz][ny][nx] arrays with x fastest.  Images are FP32
 *     or BF16 (lmr_dtype); fields are FP32 [3][nz][ny][nx] where component
 *     0/1/2 is the displacement along x/y/z in voxel units.
 *   - Pointers named as device pointers are caller-owned device memory of the
 *     current HIP device; the library never frees or retains them beyond the
 *     call (a context keeps no pointer to caller images between calls).
 *   - Work is enqueued on the stream the context (or the call) is bound to and
 *     returns without synchronising, except where a call says it synchronises.
 *   - Every call returns an lmr_status.  Invalid arguments give LMR_EINVAL and
 *     enqueue nothing.  A failing HIP runtime call gives LMR_EHIP (the HIP
 *     error string is kept, see lmr_last_error).  Asynchronous kernel faults
 *     surface at the next synchronising call.  No exception or abort crosses
 *     this interface.
 *   - A context is bound to one stream and is not re-entrant; separate
 *     contexts may be used concurrently from different threads.
 */
#ifndef LMREG_H
#define LMREG_H

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LMR_VERSION_MAJOR 0
#define LMR_VERSION_MINOR 2

typedef enum {
  LMR_OK = 0,
  LMR_EINVAL = 1,   /* invalid argument (shape, pointer, parameter) */
  LMR_ENOMEM = 2,   /* device allocation failed */
  LMR_EHIP = 3,     /* a HIP runtime call failed */
  LMR_ESTATE = 4,   /* call out of order (e.g. lmr_step before lmr_begin) */
  LMR_ESTALLED = 5, /* the pair is frozen (see lmr_params.max_retries) */
  LMR_EBUSY = 6     /* a batched launch could not have all its blocks on the GPU
                       at once (other work held it): see lmr_batch_sync */
} lmr_status;

typedef enum { LMR_F32 = 0, LMR_BF16 = 1 } lmr_dtype;

/* Accumulator of the LNCC box sums (forward, backward and the fixed image's
 * statistics).  LMR_ACC_F64: exact FP32 products summed in FP64 (default: on
 * gfx950 an FP64 add issues at the rate of an unpacked FP32 add).
 * LMR_ACC_F32C: compensated FP32, sums kept as hi/lo float pairs by cascaded
 * summation (TwoSum on the high parts, the rounding errors collected in the
 * low parts) with exact FMA products; the window statistics are then
 * formed in FP64 from hi + lo.  Both are available to every entry point,
 * the batched form included. */
typedef enum { LMR_ACC_F64 = 0, LMR_ACC_F32C = 1 } lmr_accum;

/* The optimizer of a context.  LMR_OPT_LM: the factored LM attempt (steps
 * 1-5 above).  LMR_OPT_ADAM: the paper's baseline, Adam (Sec. 3, beta1 0.9,
 * beta2 0.999) in the same kernels: the step is
 *   du = -adam_lr mhat / (sqrt(vhat) + adam_eps)
 * from bias-corrected moments of the smoothed gradient, integrated by
 * eq. compositive like the LM step, and every step is kept (no damping, no
 * rejection).  The moments add two FP32 fields (24 bytes per voxel) to the
 * workspace: the memory the paper's Sec. 3.5 compares. */
typedef enum { LMR_OPT_LM = 0, LMR_OPT_ADAM = 1 } lmr_optimizer;

/* The similarity and its least-squares residual (Sec. 2.2).
 * LMR_SIM_LNCC: L = -LNCC, r = 1 - LNCC (steps 1-5 above).
 * LMR_SIM_MSE: L = mean (F - M o (Id + u))^2, already a squared loss: the
 *   scalar residual is r = sqrt(L), the gradient g = N dr/du =
 *   (Mw - F) grad Mw / r, smoothed and used as in step 1.
 * LMR_SIM_DEMONS: the per-voxel form of the step on the squared error
 *   (Sec. 2.3, eq. demons): du_x = r_x n_x / (|n_x|^2 + lambda) with
 *   r_x = F(x) - M(x + u(x)) and n_x = grad M at x + u(x) of the accepted
 *   field, lambda global and adapted by the same rules; the step field is
 *   Gaussian-smoothed (grad_sigma) before eq. compositive.  LM only, tile 1.
 * LMR_SIM_MI: mutual information of a mi_bins x mi_bins joint histogram with
 *   cubic B-spline Parzen windows, each image mapped to bin coordinates
 *   1 + (B - 3)(v - lo)/(hi - lo) over its range (the moving range extended
 *   to 0); L = -MI (bits), r = log2 B - MI, g = N dr/du.  The histogram is
 *   summed in fixed point (2^-32), so results do not depend on the order of
 *   the additions.
 * The loss of the decision is the similarity's L in every case. */
typedef enum {
  LMR_SIM_LNCC = 0,
  LMR_SIM_MSE = 1,
  LMR_SIM_DEMONS = 2,
  LMR_SIM_MI = 3
} lmr_similarity;

/* How the three stencil passes (LNCC forward and backward, Gaussian) tile
 * the volume.  LMR_STENCIL_MARCH: 32 x 8 columns marching through chunks of
 * z planes (large volumes).  LMR_STENCIL_CUBE: 8^3 cubes of outputs, each
 * reduced along z, y and x in three steps (small volumes, where a march is
 * latency).  LMR_STENCIL_AUTO (default): cubes up to 2^20 voxels, else the
 * march.  The two forms sum the same terms in different orders (FP64 or
 * compensated sums either way). */
typedef enum {
  LMR_STENCIL_AUTO = 0,
  LMR_STENCIL_MARCH = 1,
  LMR_STENCIL_CUBE = 2
} lmr_stencil_form;

/* Hyper-parameters of one registration.  The paper's own setting
 * (Sec. 3: lambda0 = 0.006, mu+ = 1.5, mu- = 0.975, no rejection) and the
 * synthetic-phantom setting (lambda x2 / x0.5, rejection with tau = 0) are
 * both expressible; lmr_default_params fills the latter. */
typedef struct {
  int    window;       /* LNCC box side w: odd, 3..9 */
  double grad_sigma;   /* Gaussian sigma (voxels) on the gradient, 0..2; 0 = off.
                          Taps k in [-R, R], R = ceil(3 sigma), zero padding */
  double cc_eps;       /* guard added to the LNCC denominator (>= 0) */
  double step_eps;     /* eps of eq. compositive (> 0) */
  int    compositive;  /* 1: eq. compositive; 0: additive u + eps du */
  int    accum;        /* lmr_accum of the box sums */
  double lambda_inc;   /* mu+ > 1 */
  double lambda_dec;   /* 0 < mu- < 1 */
  double lambda_min;   /* lower clamp of lambda (> 0) */
  double lambda_max;   /* cap of lambda (Sec. 3.4); may be +inf */
  double tau;          /* rejection tolerance (eq. rejection); < 0 disables */
  int    max_retries;  /* consecutive rejections at lambda_max that freeze the pair */
  int    tile;         /* side k of the tiles over which the rank-1 products are
                          pooled (Sec. 2.2, eq. tilen; Sec. 3.2): each voxel
                          solves (H_tile + lambda I) du = -r g with H_tile the
                          mean of g g^T over its tile (disjoint k^3 blocks from
                          the origin); 1 (default) = eq. tile1.  1..16 */
  int    optimizer;    /* lmr_optimizer; LMR_OPT_ADAM requires tile = 1 */
  double adam_lr;      /* Adam step length in voxels (> 0; default 0.1) */
  double adam_beta1;   /* Adam decays, 0 <= beta < 1 (default 0.9, 0.999) */
  double adam_beta2;
  double adam_eps;     /* > 0 (default 1e-8) */
  int    similarity;   /* lmr_similarity (default LMR_SIM_LNCC) */
  int    mi_bins;      /* bins per image of LMR_SIM_MI, 8..32 (default 32) */
  int    stencil;      /* lmr_stencil_form (default LMR_STENCIL_AUTO) */
} lmr_params;

/* The whole optimizer state of one pair: the scalar damping and the loss
 * history that the rejection test needs (Sec. 2.2). */
typedef struct {
  double    lambda;     /* damping of the next attempt */
  double    loss;       /* L of the accepted field (L^(t-1) for the next candidate) */
  double    loss_prev;  /* L of the field accepted before it (L^(t-2)) */
  double    cand_loss;  /* L of the last candidate */
  int32_t   n_hist;     /* accepted losses recorded (1 after lmr_begin) */
  int32_t   retries;    /* consecutive rejections */
  int32_t   accepted;   /* decision of the last attempt (1 accept, 0 reject) */
  int32_t   stalled;    /* 1 once the pair is frozen */
  int64_t   attempts;   /* attempts evaluated since lmr_begin */
} lmr_pair_state;

typedef struct lmr_ctx lmr_ctx;

/* ------------------------------------------------------------------------ */
const char* lmr_strerror(lmr_status s);
/* Text of the last HIP error seen by this thread (empty if none). */
const char* lmr_last_error(void);
void lmr_default_params(lmr_params* p);

/* Creates a context for one pair (the state the paper's optimizer keeps per
 * pair: the field and the scalar damping with its loss history, Sec. 2.2)
 * for volumes of nz*ny*nx voxels with images of type img,
 * bound to `stream` (0 = the null stream).  Allocates the whole workspace
 * (about 80 bytes per voxel: field ping-pong, smoothed gradient, raw
 * gradient, four LNCC adjoint maps, warped image, reduction partials and the
 * device pair state); no later call allocates.  Sizes: each dimension >= 1,
 * nz*ny*nx < 2^30 (kernels address each channel with 32-bit byte offsets).
 * Errors: LMR_EINVAL (shape/params), LMR_ENOMEM. */
lmr_status lmr_create(lmr_ctx** out, int nz, int ny, int nx, lmr_dtype img,
                      const lmr_params* p, hipStream_t stream);
void lmr_destroy(lmr_ctx* ctx);

/* Starts a registration from `field` (device, [3][nz][ny][nx] FP32; NULL =
 * identity u = 0) with damping lambda0 > 0: evaluates L(u) and the smoothed
 * gradient of u (the Eulerian descent direction, Sec. 2.1; the residual
 * r = 1 - LNCC of Sec. 2.2).  fixed/moving: device images of the context's type.  The
 * window mean and variance of `fixed`, which no attempt changes, are computed
 * here once and kept in the context. */
lmr_status lmr_begin(lmr_ctx* ctx, const void* fixed, const void* moving,
                     const float* field, double lambda0);

/* Enqueues n_attempts LM attempts (steps 1-5 above).  Each attempt reads the
 * accepted field, its smoothed gradient and (lambda, r) from device memory
 * and leaves the decision there; nothing returns to the host, so the calls
 * may be captured in a HIP graph.  A frozen pair skips its work.  The window
 * statistics of `fixed` are reused from lmr_begin while the same buffer is
 * passed (another buffer makes the call recompute them first; contents
 * changed in place need a new lmr_begin).
 * Errors: LMR_ESTATE before lmr_begin. */
lmr_status lmr_step(lmr_ctx* ctx, const void* fixed, const void* moving,
                    int n_attempts);

/* As lmr_step, with the accept/reject decision of attempt i forced to
 * decisions[i] (host array; 1 accept, 0 reject, -1 automatic).  Lambda and
 * the loss history follow the forced decision exactly as they would follow
 * an automatic one.  Used to replay a recorded trajectory.  An Adam context
 * keeps every step: a forced rejection gives LMR_EINVAL. */
lmr_status lmr_step_forced(lmr_ctx* ctx, const void* fixed, const void* moving,
                           const int* decisions, int n);
/* Forces the decision of every later lmr_step attempt (1 accept, 0 reject,
 * -1 automatic, the default) until called again; lambda and the loss history
 * follow a forced decision as they follow an automatic one (Sec. 2.2,
 * eq. lambda-update; Sec. 3.4, eq. rejection).  LMR_EINVAL for other values,
 * and for 0 on an Adam context. */
lmr_status lmr_force_decision(lmr_ctx* ctx, int decision);

/* Bytes of device memory the context holds (its whole workspace). */
lmr_status lmr_workspace_bytes(const lmr_ctx* ctx, size_t* out);

/* Copies the accepted field u (Sec. 2.1: the displacement of Id + u, voxel
 * units) into field_out (device, [3][nz][ny][nx]). */
lmr_status lmr_get_field(lmr_ctx* ctx, float* field_out);
/* Copies the smoothed gradient of the accepted field (Sec. 2.1) into g_out
 * (device). */
lmr_status lmr_get_grad(lmr_ctx* ctx, float* g_out);
/* Synchronises the context's stream and returns the pair state (lambda and
 * the loss history of Sec. 2.2 and Sec. 3.4). */
lmr_status lmr_get_state(lmr_ctx* ctx, lmr_pair_state* out);
/* Overwrites the device pair state with `in` (host struct): lambda, the loss
 * history, counters and flags.  With lmr_begin on a saved field this resumes
 * a registration from a checkpoint (lmr_get_field + lmr_get_state); the
 * resumed attempts are bitwise identical to the uninterrupted ones when `in`
 * holds the saved state.  Requires lambda > 0 and n_hist >= 1.  Asynchronous
 * (the struct is copied before the call returns).  LMR_EINVAL on an Adam
 * context (its moments are part of its state and are not restored here). */
lmr_status lmr_set_state(lmr_ctx* ctx, const lmr_pair_state* in);

/* Test hook: loss and gradients of an arbitrary field u (device) without
 * touching the pair state.  loss_out (host) receives L = -mean cc; g_raw and
 * g_smooth (device, [3][nz][ny][nx], either may be NULL) receive N dL/du and
 * its Gaussian-smoothed version; cc_map (device [nz][ny][nx], may be NULL)
 * receives cc(x).  Synchronises. */
lmr_status lmr_loss_grad(lmr_ctx* ctx, const void* fixed, const void* moving,
                         const float* u, double* loss_out, float* g_raw,
                         float* g_smooth, float* cc_map);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * results of lmr_loss_grad without a context and without any allocation.
 * F, M: device images of type img, [nz][ny][nx]; u: device field
 * [3][nz][ny][nx]; p: the parameters (window, grad_sigma, cc_eps, accum are
 * used); loss_dev: device double receiving L = -mean cc; g_raw, g_smooth
 * (device [3][nz][ny][nx], either may be NULL, not the same buffer) and
 * cc_map (device [nz][ny][nx], may be NULL) as in lmr_loss_grad.  The
 * results are bitwise those of lmr_loss_grad on the same inputs.
 * Enqueues on `stream` and returns without synchronising.
 * Workspace: one static device array of this library (about 48 MiB, held
 * by every GPU the library runs on until the process ends), so volumes are
 * limited to nz*ny*nx <= 2^20 voxels; larger ones give LMR_EINVAL.  Every
 * call on a GPU uses that GPU's one array: calls that overlap on one GPU
 * (different streams or threads) race and must be serialised by the
 * caller.  Nothing in it needs clearing between calls (each call writes
 * every value it reads). */
lmr_status lmr_loss_grad_noalloc(const void* fixed, const void* moving, lmr_dtype img,
                                 const float* u, int nz, int ny, int nx,
                                 const lmr_params* p, double* loss_dev, float* g_raw,
                                 float* g_smooth, float* cc_map, hipStream_t stream);

/* Test hook: steps 1-2 alone.  u_out = eps du + u o (Id + eps du) with
 * du = -r g / (|g|^2 + lambda) (device arrays, [3][nz][ny][nx]), or with
 * tile > 1 du = -r (H_tile + lambda I)^-1 g, H_tile pooled from g_smooth
 * (the context's tile workspace is overwritten).  LMR_EINVAL on an Adam
 * context. */
lmr_status lmr_update(lmr_ctx* ctx, const float* u, const float* g_smooth,
                      double r, double lambda, float* u_out);

/* Folded-voxel count: the number of voxels where det(I + grad u) <= 0, with
 * central differences inside the volume and first-order one-sided differences
 * on its faces (the folding test that judges a deformation; used by the
 * learned initializer's gate).  u: device field, or NULL for the context's
 * accepted field (then the raw-gradient workspace is overwritten).  det_out
 * (device [nz][ny][nx], may be NULL) receives det(I + grad u) rounded to
 * FP32; the decision is taken in FP64.  Synchronises. */
lmr_status lmr_folded_count(lmr_ctx* ctx, const float* u, long long* count_out,
                            float* det_out);

/* Gaussian smoothing of a field (step 5 alone): out = G_sigma * g with the
 * context's grad_sigma, taps k in [-R, R], R = ceil(3 sigma), zero padding
 * (Eulerian descent, Sec. 2.1).  g and out: device [3][nz][ny][nx], distinct. */
lmr_status lmr_smooth(lmr_ctx* ctx, const float* g, float* out);

/* Test hook: step 4 alone.  Runs the device decision once on the state
 * `in` with candidate loss cand_loss and forced decision `force` (-1
 * automatic, 0 reject, 1 accept), and returns the resulting state in `out`
 * (host structs).  Uses a private device state: the context's pair state is
 * untouched.  Synchronises. */
lmr_status lmr_decide_probe(lmr_ctx* ctx, const lmr_pair_state* in,
                            double cand_loss, int force, lmr_pair_state* out);

/* ------------------------------------------------------------------------ */
/* Kernel timing.  While a profile is open, lmr_step records HIP events on
 * the context's stream in every `stride`-th attempt (at most max_attempts
 * attempts): one before its first kernel and one after each kernel, so that
 * a kernel's duration runs from the end of the one before it (its launch gap
 * included) to its own end.  lmr_profile_stop synchronises and returns
 * per-kernel count and duration statistics indexed by lmr_kernel. */
typedef enum {
  LMR_K_UPDATE = 0,  /* closed form + compositive integration + candidate warp */
  LMR_K_FWD = 1,     /* LNCC forward (box sums, cc, adjoint maps, partials) */
  LMR_K_DECIDE = 2,  /* FP64 loss reduction and decision (LNCC levels with at most
                        1024 partials and a window of at most 7, marching or on
                        4-plane bricks, take it inside the backward pass: this
                        interval is then its event alone) */
  LMR_K_BWD = 3,     /* LNCC backward and warp backward */
  LMR_K_SMOOTH = 4,  /* Gaussian smoothing of the gradient */
  LMR_NUM_KERNELS = 5
} lmr_kernel;
typedef struct {
  int64_t count;
  double total_ms, min_ms, max_ms;
} lmr_kernel_time;
lmr_status lmr_profile_start(lmr_ctx* ctx, int max_attempts, int stride);
lmr_status lmr_profile_stop(lmr_ctx* ctx, lmr_kernel_time out[LMR_NUM_KERNELS]);
const char* lmr_kernel_name(int kernel);

/* ------------------------------------------------------------------------ */
/* Coarse-to-fine registration (Sec. 2.1): level l works on images average-
 * pooled by factors[l] (coarse to fine, each factor twice the next, the last
 * one 1, every dimension divisible by factors[0]); level 0 starts from the
 * identity, every later level from the previous field upsampled x2 (voxel-
 * centre aligned, values doubled).  Lambda and the loss history restart at
 * every level (losses of different resolutions are not comparable).  All
 * level workspaces and pooled images (FP32) are allocated here. */
typedef struct lmr_pyramid lmr_pyramid;
lmr_status lmr_pyramid_create(lmr_pyramid** out, int nz, int ny, int nx,
                              lmr_dtype img, const lmr_params* p, int nlevels,
                              const int* factors, hipStream_t stream);
/* Runs iters[l] attempts at every level (host array of nlevels counts) from
 * lambda0 and writes the final field (device, [3][nz][ny][nx]).  decisions:
 * NULL for automatic decisions, or a host array of sum(iters) forced
 * decisions (level-major).  Enqueues only. */
lmr_status lmr_pyramid_run(lmr_pyramid* pyr, const void* fixed, const void* moving,
                           const int* iters, double lambda0, const int* decisions,
                           float* field_out);
/* Automatic attempts of a level run as one HIP graph launch per level
 * (captured on first use for the given images and attempt count, on a
 * private stream, and replayed on the pyramid's stream; the images must stay
 * at the same addresses for a replay to apply).  enable = 0 enqueues the
 * attempts one kernel at a time instead.  Default: enabled.  Forced decisions
 * run eagerly.  On a level whose kernel timing is open with stride 1 every
 * attempt runs eagerly; with stride s > 1 the sampled attempts run eagerly
 * between their events and the s - 1 attempts between two samples as one
 * graph launch (captured with the profiler off). */
lmr_status lmr_pyramid_use_graphs(lmr_pyramid* pyr, int enable);
/* The context of level l (borrowed; valid until lmr_pyramid_destroy). */
lmr_ctx* lmr_pyramid_level(lmr_pyramid* pyr, int level);
void lmr_pyramid_destroy(lmr_pyramid* pyr);

/* ------------------------------------------------------------------------ */
/* Batched form: npairs pairs of uneven shapes (shapes: host array of npairs
 * triples nz, ny, nx) advance together, each with its own lambda, loss
 * history and decision.  An attempt of all pairs runs phase by phase
 * (update, LNCC forward, decision, LNCC backward, smoothing) over the work
 * items of all pairs, either as one launch per phase (the default) or as ONE
 * persistent launch per attempt: a grid of as many blocks as fit on the GPU
 * at once sweeps the items with a grid barrier between phases
 * (lmr_batch_set_config; both give the same results bit for bit).  The
 * launches of lmr_batch_step are captured in a HIP graph on first use and
 * replayed.  The batch owns a non-blocking stream; results of one pair are
 * read through lmr_batch_pair (borrowed context).  Box side 3..9 and
 * Gaussian radius ceil(3 sigma) <= 4 are supported (else LMR_EINVAL).  A pair
 * that a stand-alone context with p->stencil runs on 4-plane bricks runs on
 * the same bricks here; the others march (LMR_STENCIL_MARCH); either way a
 * pair follows the stand-alone context with that form bit for bit.
 *
 * Co-residency (persistent launches only).  The persistent launch needs all
 * its blocks on the GPU at once; the caller must not run other kernels at
 * the same time on other streams (another batch's steps included) that could
 * hold the resources some of its blocks need.  Each launch checks this at its
 * first barrier: when a block has waited there 2 ms while some block of the
 * grid has not even started, the launch gives up and lmr_batch_sync reports
 * LMR_EBUSY (a few milliseconds, not a timeout): the pairs keep the state of
 * the last completed launch, later launches of the same step return at once,
 * and the batch may be stepped again once the other work is done.  Any
 * barrier wait longer than 0.25 s also makes every block leave (LMR_EHIP at
 * lmr_batch_sync).  Neither can hang the device.  One launch per phase has no
 * such requirement. */
typedef struct lmr_batch lmr_batch;
lmr_status lmr_batch_create(lmr_batch** out, int npairs, const int* shapes,
                            lmr_dtype img, const lmr_params* p);
/* Starts every pair from the identity with lambda0[i] (NULL: 1.0).  fixed[i],
 * moving[i]: device images of pair i, which must stay valid while the batch
 * steps (the batched kernels read them through a device table).  Returns
 * after the batch stream has finished this work. */
lmr_status lmr_batch_begin(lmr_batch* b, const void* const* fixed,
                           const void* const* moving, const double* lambda0);
/* Enqueues n_iters iterations (one persistent launch, or one launch per
 * phase, each); use_graph = 1 replays a captured HIP graph of them. */
lmr_status lmr_batch_step(lmr_batch* b, int n_iters, int use_graph);
/* Synchronises the batch stream; LMR_EBUSY if a launch was not co-resident,
 * LMR_EHIP if a barrier wait timed out (both clear, so the batch can go on). */
lmr_status lmr_batch_sync(lmr_batch* b);
/* For callers testing their handling of LMR_EBUSY: with late_block = 1, block
 * 0 of every later launch starts 4 ms late, as a block that was not on the
 * GPU would, so each launch takes the co-residency failure path above
 * (0 = normal operation, the default). */
lmr_status lmr_batch_test_residency(lmr_batch* b, int late_block);
lmr_ctx* lmr_batch_pair(lmr_batch* b, int i);
/* Tiling knobs: target tile count per pair (0, the default: each pair tiled
 * as a stand-alone context's marching passes tile it, so that a pair's run
 * is bit for bit the per-pair run; else 64 ... 2^20), minimum z-chunk (4 ...
 * 256; unused with target 0), persistent blocks per CU (-1, the default:
 * no persistent kernel, each phase of an attempt is one launch over the work
 * items of all pairs, the same items and results, 5 to 8 launches per
 * attempt, and no co-residency requirement; 0 = one persistent launch per
 * attempt with as many blocks as fit; n > 0 = n blocks per CU).  Pairs that a stand-alone context runs on 4-plane bricks run on
 * the same bricks here (either mode); the others march. */
lmr_status lmr_batch_set_config(lmr_batch* b, int target_tiles, int min_cz,
                                int blocks_per_cu);
lmr_status lmr_batch_get_config(lmr_batch* b, int cfg[3]);
/* Autotuner: times iters_per_trial iterations for every candidate
 * configuration on the given images and keeps the fastest; with cache_path
 * the choice is read from / appended to that text file, keyed by the GPU,
 * image type, window, sigma and the pair shapes.  best_ms (may be NULL)
 * receives the time of one iteration.  The trials overwrite the pair states:
 * call lmr_batch_begin afterwards. */
lmr_status lmr_batch_tune(lmr_batch* b, const void* const* fixed,
                          const void* const* moving, const char* cache_path,
                          int iters_per_trial, double* best_ms);
void lmr_batch_destroy(lmr_batch* b);

/* Average pooling by f (every dimension divisible by f): out (device, FP32,
 * [nz/f][ny/f][nx/f]) is the mean of each f^3 block of img. */
lmr_status lmr_avgpool(const void* img, lmr_dtype t, int nz, int ny, int nx, int f,
                       float* out, hipStream_t stream);
/* x2 field upsampling of the pyramid: uc [3][nzc][nyc][nxc] ->
 * uf [3][2nzc][2nyc][2nxc] (device). */
lmr_status lmr_upsample_field(const float* uc, int nzc, int nyc, int nxc, float* uf,
                              hipStream_t stream);

/* Trilinear warp Mw(x) = M(x + u(x)), zero outside the volume; dMw (may be
 * NULL) receives d/dp M at x + u(x) as [3][nz][ny][nx].  Device arrays. */
lmr_status lmr_warp(const void* moving, lmr_dtype img, const float* u,
                    int nz, int ny, int nx, float* Mw, float* dMw,
                    hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* LMREG_H */
