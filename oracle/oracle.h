/*
 * FP64 CPU oracle for the factored Levenberg-Marquardt registration step.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and oracle.c exist to check the GPU
 * library against a plain, slow, obviously correct re-statement of the method
 * ("Factored Levenberg-Marquardt for Diffeomorphic Image Registration",
 * arXiv 2603.19371).  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source, header, table or
 * helper with the GPU library (paper_2603_19371_amd/csrc, include/lmreg.h).
 *
 * Conventions (all arrays host memory, double precision):
 *   volume   V[z][y][x], x fastest;  N = nz*ny*nx;  idx = (z*ny + y)*nx + x
 *   field    u[c][z][y][x], c = 0,1,2 holds the displacement along x,y,z in
 *            voxel units (a point x is mapped to x + u(x)).
 *   window   LNCC box side w (odd), half-width h = w/2, n = w^3.
 */
#ifndef LMR_ORACLE_H
#define LMR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Parameters of one registration (Sec. 2.2 and Sec. 3.4 of the paper). */
typedef struct {
  int    window;       /* LNCC box side w, odd, >= 1 */
  double grad_sigma;   /* Gaussian sigma applied to the gradient; 0 = none */
  double cc_eps;       /* guard added to the LNCC denominator */
  double step_eps;     /* epsilon of the compositive update (Sec. 2.1) */
  int    compositive;  /* 1: compositive update, 0: additive u + eps v */
  double lambda_inc;   /* mu+ > 1 (eq. lambda-update) */
  double lambda_dec;   /* 0 < mu- < 1 (eq. lambda-update) */
  double lambda_min;   /* lower clamp of lambda */
  double lambda_max;   /* cap of lambda (Sec. 3.4) */
  double tau;          /* rejection tolerance (eq. rejection); < 0 disables */
  int    max_retries;  /* consecutive rejections before a pair is frozen */
  int    tile;         /* tile side k of the pooled Hessian (eq. tilen); 1 = eq. tile1 */
  int    similarity;   /* 0 LNCC, 1 squared error (MSE), 2 Demons step on the MSE,
                          3 mutual information */
  int    mi_bins;      /* B, the Parzen histogram's bins per image (>= 4) */
} orc_params;

/* Hyper-parameters of the Eulerian Adam comparator (the paper's baseline
 * optimizer, Sec. 3: beta1 = 0.9, beta2 = 0.999). */
typedef struct {
  double lr;     /* step length eta in voxels */
  double beta1;  /* first-moment decay */
  double beta2;  /* second-moment decay */
  double eps;    /* added to the root of the second moment */
} orc_adam_params;

/* Whole optimizer state of one pair: the scalar damping and a short loss
 * history (Sec. 2.2, "LM with rejection criterion"). */
typedef struct {
  double lambda;     /* damping used by the next attempt */
  double loss;       /* L of the accepted field  (= L^(t-1) for a candidate) */
  double loss_prev;  /* L of the field accepted before it (= L^(t-2)) */
  double cand_loss;  /* L of the last candidate */
  int    n_hist;     /* number of accepted losses recorded (1 after begin) */
  int    retries;    /* consecutive rejections */
  int    accepted;   /* decision of the last attempt */
  int    stalled;    /* 1 once the pair is frozen */
} orc_state;

/* O1: trilinear sample of V at (px,py,pz), zero outside; dv (may be NULL)
 * receives d/dp of the interpolant on the cell [floor(p), floor(p)+1]. */
double orc_sample(const double* V, int nz, int ny, int nx,
                  double px, double py, double pz, double* dv);
/* O1: Mw(x) = M(x + u(x)); dMw[c][x] (may be NULL) = d/dp_c M at x + u(x). */
void orc_warp(const double* M, const double* u, int nz, int ny, int nx,
              double* Mw, double* dMw);

/* O2: zero-padded box sum over the w^3 window centred at each voxel. */
void orc_box_sum(const double* a, int nz, int ny, int nx, int w, double* out);
/* O2: local statistics at one voxel (definition, brute force). */
void orc_window_stats(const double* F, const double* Mw, int nz, int ny, int nx,
                      int w, int x, int y, int z, double st[5]);
/* O2: LNCC map cc[N] (may be NULL); returns the mean of cc over the volume. */
double orc_lncc(const double* F, const double* Mw, int nz, int ny, int nx,
                int w, double eps, double* cc);
/* O3: dS[j] = d(sum_x cc(x)) / d Mw_j  (chain rule over every window that
 * contains j). */
void orc_dsumcc_dmw(const double* F, const double* Mw, int nz, int ny, int nx,
                    int w, double eps, double* dS);
/* O2+O3: loss L = -mean cc of (F, M o (Id+u)) and g_raw = N * dL/du. */
double orc_loss_grad(const double* F, const double* M, const double* u,
                     int nz, int ny, int nx, int w, double eps, double* g_raw);
/* O3 at one voxel j only: g_raw[3] at (x,y,z).  Evaluates only the windows
 * that reach j, so it can be used on large volumes. */
void orc_grad_at(const double* F, const double* M, const double* u,
                 int nz, int ny, int nx, int w, double eps,
                 int x, int y, int z, double g[3]);

/* Squared error (Sec. 2.2: already a squared loss): L = mean (F - Mw)^2 and
 * g_raw = N dr/du with the scalar residual r = sqrt(L) (0 where r = 0). */
double orc_mse_loss_grad(const double* F, const double* M, const double* u,
                         int nz, int ny, int nx, double* g_raw);
/* Mutual information (Sec. 2.2: minimise (log2 B - MI)^2) of F and
 * M o (Id + u) from a joint histogram of B x B bins with cubic B-spline
 * Parzen windows.  Each image's values are mapped to bin coordinates
 * 1 + (B - 3)(v - lo)/(hi - lo) with [lo, hi] its range over the volume
 * (the moving range extended to 0, the value outside the volume).
 * Returns L = -MI (bits); g_raw (may be NULL) = N dr/du, r = log2 B - MI;
 * hist (may be NULL) receives the joint probabilities [B][B] (fixed bin
 * major). */
double orc_mi_loss_grad(const double* F, const double* M, const double* u, int nz,
                        int ny, int nx, int B, double* g_raw, double* hist);
/* Cubic B-spline and its derivative (the Parzen window). */
double orc_bspline3(double t);
double orc_dbspline3(double t);

/* Demons step (Sec. 2.3, eq. demons): du_x = r_x n_x / (|n_x|^2 + lambda)
 * with r_x = F - M o (Id + u) and n_x = grad M at x + u(x). */
void orc_demons_step(const double* F, const double* M, const double* u, int nz,
                     int ny, int nx, double lambda, double* du);

/* O2 at one voxel: cc(x) of (F, M o (Id + u)), warping only the window. */
double orc_cc_at(const double* F, const double* M, const double* u, int nz,
                 int ny, int nx, int w, double eps, int x, int y, int z);

/* O4: 3D Gaussian of nc channels, taps k in [-R,R], R = ceil(3 sigma),
 * zero outside, weights normalised over the full tap range. */
void orc_gauss(const double* g, int nc, int nz, int ny, int nx, double sigma,
               double* out);
int  orc_gauss_radius(double sigma);
/* O4 at one voxel, nc channels. */
void orc_gauss_at(const double* g, int nc, int nz, int ny, int nx, double sigma,
                  int x, int y, int z, double* out);

/* O5: closed-form damped rank-1 step (eq. tile1). */
void orc_closed_form(const double* gs, int nz, int ny, int nx, double r,
                     double lambda, double* du);
/* O5 check: explicit 3x3 solve (g g^T + lambda I) d = -r g by Gaussian
 * elimination with partial pivoting (eq. lm-local). */
void orc_explicit_solve(const double g[3], double r, double lambda, double d[3]);

/* O5' (eq. tilen): pooled Hessian of tile side k.  Tiles are the disjoint
 * k^3 blocks of the grid starting at the origin (partial blocks at the far
 * faces); H[t][6] = mean over the voxels of tile t of gs gs^T, entries
 * (xx, yy, zz, xy, xz, yz).  Tiles are numbered x fastest. */
void orc_tile_hessian(const double* gs, int nz, int ny, int nx, int k, double* H);
/* O5' step: for every voxel, (H_tile + lambda I) du = -r gs by Gaussian
 * elimination with partial pivoting (k = 1 gives eq. tile1). */
void orc_tile_step(const double* gs, int nz, int ny, int nx, int k, double r,
                   double lambda, double* du);

/* Adam comparator: one bias-corrected Adam direction on gs at step t >= 1.
 * m, v (3N) are updated in place; du = -lr mhat / (sqrt(vhat) + eps). */
void orc_adam_direction(const double* gs, double* m, double* v, long n, long t,
                        const orc_adam_params* a, double* du);

/* O6: u_new = eps v + u o (Id + eps v)  (eq. compositive), or u + eps v. */
void orc_integrate(const double* u, const double* v, int nz, int ny, int nx,
                   double eps, int compositive, double* unew);

/* O7: decision on a candidate loss (eq. lambda-update, eq. rejection).
 * force: -1 automatic, 0 reject, 1 accept.  Returns 1 if accepted. */
int orc_decide(const orc_params* p, orc_state* s, double cand_loss, int force);

/* One registration pair: evaluates L(u) and the smoothed gradient of u. */
void orc_begin(const orc_params* p, const double* F, const double* M,
               const double* u, int nz, int ny, int nx, double lambda0,
               orc_state* s, double* gs_out);
/* One LM attempt.  u and gs hold the accepted field and its smoothed gradient
 * and are replaced on acceptance.  Returns the decision. */
int orc_attempt(const orc_params* p, const double* F, const double* M,
                double* u, double* gs, int nz, int ny, int nx,
                orc_state* s, int force);

/* One iteration of the Adam comparator: du from the moments of gs (step t),
 * u <- eps du + u o (Id + eps du), then the loss and the smoothed gradient
 * of the new field.  Every iteration is kept (no damping, no rejection);
 * s->loss and s->cand_loss receive the new loss. */
void orc_adam_iter(const orc_params* p, const orc_adam_params* a, const double* F,
                   const double* M, double* u, double* gs, double* m, double* v,
                   int nz, int ny, int nx, long t, orc_state* s);

/* O8: average pooling by an integer factor (each dim divisible). */
void orc_avgpool(const double* a, int nz, int ny, int nx, int f, double* out);
/* O8: field upsampling x2, voxel-centre aligned, values doubled. */
void orc_upsample_field(const double* uc, int nzc, int nyc, int nxc,
                        double* uf, int nz, int ny, int nx);

/* O9: number of voxels with det(I + grad u) <= 0. */
long orc_folded_count(const double* u, int nz, int ny, int nx, double* det);

#ifdef __cplusplus
}
#endif
#endif
