/*
 * FP64 CPU oracle for the factored Levenberg-Marquardt registration step
 * (arXiv 2603.19371).  TEST INFRASTRUCTURE ONLY: it is loaded by the tests,
 * the smoke check and the CPU-baseline leg of the benchmark, never by the
 * product path.  It shares no code with the GPU library.
 *
 * Every function is the plain definition of what it computes, in double
 * precision, with no blocking, no separable passes, no sliding windows and
 * no fusion: box sums and the Gaussian are evaluated tap by tap.  Where the
 * paper is silent the reading taken is stated at the function.
 *
 * Pins (tests/test_oracle_*.py) tie each function to something other than
 * itself: scipy/numpy/torch library routines, closed forms, invariants and
 * finite differences.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(z, y, x) (((long)(z) * ny + (y)) * nx + (x))

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* O1  warp M o (Id + u)  (Sec. 1, eq. 1: L_sim(F, M o phi), phi = Id + u)   */
/* ------------------------------------------------------------------------ */

/* Trilinear interpolation.  Reading: a corner outside the volume contributes
 * the value 0 (zero padding).  The derivative is that of the interpolating
 * polynomial on the cell [floor(p), floor(p)+1] along each axis, so at an
 * exactly integer coordinate it is the forward difference. */
double orc_sample(const double* V, int nz, int ny, int nx, double px,
                  double py, double pz, double* dv) {
  if (dv) dv[0] = dv[1] = dv[2] = 0.0;
  if (!(isfinite(px) && isfinite(py) && isfinite(pz))) return 0.0;
  /* far outside: every corner is padding */
  if (px < -2.0 || py < -2.0 || pz < -2.0 || px > nx + 1.0 || py > ny + 1.0 ||
      pz > nz + 1.0)
    return 0.0;
  double bx = floor(px), by = floor(py), bz = floor(pz);
  double fx = px - bx, fy = py - by, fz = pz - bz;
  long x0 = (long)bx, y0 = (long)by, z0 = (long)bz;
  double val = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int c = 0; c < 2; c++) {
    for (int b = 0; b < 2; b++) {
      for (int a = 0; a < 2; a++) {
        long xi = x0 + a, yi = y0 + b, zi = z0 + c;
        double v = 0.0;
        if (xi >= 0 && xi < nx && yi >= 0 && yi < ny && zi >= 0 && zi < nz)
          v = V[IDX(zi, yi, xi)];
        double wx = a ? fx : 1.0 - fx, dwx = a ? 1.0 : -1.0;
        double wy = b ? fy : 1.0 - fy, dwy = b ? 1.0 : -1.0;
        double wz = c ? fz : 1.0 - fz, dwz = c ? 1.0 : -1.0;
        val += wx * wy * wz * v;
        gx += dwx * wy * wz * v;
        gy += wx * dwy * wz * v;
        gz += wx * wy * dwz * v;
      }
    }
  }
  if (dv) {
    dv[0] = gx;
    dv[1] = gy;
    dv[2] = gz;
  }
  return val;
}

void orc_warp(const double* M, const double* u, int nz, int ny, int nx,
              double* Mw, double* dMw) {
  long N = (long)nz * ny * nx;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        long i = IDX(z, y, x);
        double d[3];
        Mw[i] = orc_sample(M, nz, ny, nx, x + u[i], y + u[N + i],
                           z + u[2 * N + i], dMw ? d : NULL);
        if (dMw) {
          dMw[i] = d[0];
          dMw[N + i] = d[1];
          dMw[2 * N + i] = d[2];
        }
      }
}

/* ------------------------------------------------------------------------ */
/* O2  LNCC forward (Sec. 2.2 item 2: minimise (1 - LNCC)^2; Sec. 3 uses the */
/*     fused local cross-correlation).  The paper prints no formula; the      */
/*     reading is the windowed squared correlation below.                    */
/* ------------------------------------------------------------------------ */

/* Box sum over the w^3 window centred at each voxel.  Reading: voxels outside
 * the volume count as zero and the divisor used by the statistics stays
 * n = w^3 at every centre. */
void orc_box_sum(const double* a, int nz, int ny, int nx, int w, double* out) {
  int h = w / 2;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        double s = 0.0;
        for (int dz = -h; dz <= h; dz++)
          for (int dy = -h; dy <= h; dy++)
            for (int dx = -h; dx <= h; dx++) {
              int zz = z + dz, yy = y + dy, xx = x + dx;
              if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx)
                continue;
              s += a[IDX(zz, yy, xx)];
            }
        out[IDX(z, y, x)] = s;
      }
}

/* Sums S_F, S_M, S_FF, S_MM, S_FM over the window centred at (x,y,z). */
void orc_window_stats(const double* F, const double* Mw, int nz, int ny,
                      int nx, int w, int x, int y, int z, double st[5]) {
  int h = w / 2;
  double sf = 0, sm = 0, sff = 0, smm = 0, sfm = 0;
  for (int dz = -h; dz <= h; dz++)
    for (int dy = -h; dy <= h; dy++)
      for (int dx = -h; dx <= h; dx++) {
        int zz = z + dz, yy = y + dy, xx = x + dx;
        if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx)
          continue;
        double f = F[IDX(zz, yy, xx)], m = Mw[IDX(zz, yy, xx)];
        sf += f;
        sm += m;
        sff += f * f;
        smm += m * m;
        sfm += f * m;
      }
  st[0] = sf;
  st[1] = sm;
  st[2] = sff;
  st[3] = smm;
  st[4] = sfm;
}

/* Local moments and their derivatives at one centre.
 *   mu_F = S_F/n, mu_M = S_M/n
 *   s_FM = S_FM/n - mu_F mu_M, s_FF = S_FF/n - mu_F^2, s_MM = S_MM/n - mu_M^2
 *   cc   = s_FM^2 / (s_FF s_MM + eps)
 *   alpha = d cc / d s_FM = 2 s_FM / D,  beta = d cc / d s_MM = -s_FM^2 s_FF / D^2
 * with D = s_FF s_MM + eps.  Squared correlation (so cc lies in [0,1] and is
 * insensitive to contrast polarity) is the reading taken for the unprinted
 * LNCC formula. */
typedef struct {
  double muF, muM, cc, alpha, beta;
} orc_local;

static orc_local local_from_sums(const double st[5], int w, double eps) {
  double n = (double)w * w * w;
  orc_local o;
  o.muF = st[0] / n;
  o.muM = st[1] / n;
  double sfm = st[4] / n - o.muF * o.muM;
  double sff = st[2] / n - o.muF * o.muF;
  double smm = st[3] / n - o.muM * o.muM;
  double D = sff * smm + eps;
  o.cc = sfm * sfm / D;
  o.alpha = 2.0 * sfm / D;
  o.beta = -sfm * sfm * sff / (D * D);
  return o;
}

double orc_lncc(const double* F, const double* Mw, int nz, int ny, int nx,
                int w, double eps, double* cc) {
  double total = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : total)
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        double st[5];
        orc_window_stats(F, Mw, nz, ny, nx, w, x, y, z, st);
        orc_local o = local_from_sums(st, w, eps);
        if (cc) cc[IDX(z, y, x)] = o.cc;
        total += o.cc;
      }
  return total / ((double)nz * ny * nx);
}

/* ------------------------------------------------------------------------ */
/* O3  LNCC backward: chain rule of sum_x cc(x) with respect to Mw_j.        */
/*   d s_FM(x)/d Mw_j = (F_j - mu_F(x)) / n                                  */
/*   d s_MM(x)/d Mw_j = 2 (Mw_j - mu_M(x)) / n                               */
/* for every in-volume centre x whose window holds j.                        */
/* ------------------------------------------------------------------------ */

static void local_maps(const double* F, const double* Mw, int nz, int ny,
                       int nx, int w, double eps, orc_local* L) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        double st[5];
        orc_window_stats(F, Mw, nz, ny, nx, w, x, y, z, st);
        L[IDX(z, y, x)] = local_from_sums(st, w, eps);
      }
}

static double dsum_at(const orc_local* L, const double* F, const double* Mw,
                      int nz, int ny, int nx, int w, int x, int y, int z) {
  int h = w / 2;
  double n = (double)w * w * w;
  double fj = F[IDX(z, y, x)], mj = Mw[IDX(z, y, x)];
  double s = 0.0;
  for (int dz = -h; dz <= h; dz++)
    for (int dy = -h; dy <= h; dy++)
      for (int dx = -h; dx <= h; dx++) {
        int zz = z + dz, yy = y + dy, xx = x + dx;
        if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx)
          continue;
        const orc_local* o = &L[IDX(zz, yy, xx)];
        s += o->alpha * (fj - o->muF) / n + o->beta * 2.0 * (mj - o->muM) / n;
      }
  return s;
}

void orc_dsumcc_dmw(const double* F, const double* Mw, int nz, int ny, int nx,
                    int w, double eps, double* dS) {
  long N = (long)nz * ny * nx;
  orc_local* L = (orc_local*)malloc(sizeof(orc_local) * N);
  local_maps(F, Mw, nz, ny, nx, w, eps, L);
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++)
        dS[IDX(z, y, x)] = dsum_at(L, F, Mw, nz, ny, nx, w, x, y, z);
  free(L);
}

/* Loss L = -mean_x cc(x) (Sec. 2.2: the residual is r = 1 - LNCC = 1 + L)
 * and g_raw = N dL/du.  Reading: the gradient is that of the sum-reduced
 * loss -sum cc, so that its scale does not depend on the volume size. */
double orc_loss_grad(const double* F, const double* M, const double* u,
                     int nz, int ny, int nx, int w, double eps,
                     double* g_raw) {
  long N = (long)nz * ny * nx;
  double* Mw = (double*)malloc(sizeof(double) * N);
  double* dMw = (double*)malloc(sizeof(double) * 3 * N);
  orc_warp(M, u, nz, ny, nx, Mw, dMw);
  double lncc = orc_lncc(F, Mw, nz, ny, nx, w, eps, NULL);
  if (g_raw) {
    double* dS = (double*)malloc(sizeof(double) * N);
    orc_dsumcc_dmw(F, Mw, nz, ny, nx, w, eps, dS);
    for (long i = 0; i < N; i++)
      for (int c = 0; c < 3; c++) g_raw[c * N + i] = -dS[i] * dMw[c * N + i];
    free(dS);
  }
  free(Mw);
  free(dMw);
  return -lncc;
}

void orc_grad_at(const double* F, const double* M, const double* u, int nz,
                 int ny, int nx, int w, double eps, int x, int y, int z,
                 double g[3]) {
  long N = (long)nz * ny * nx;
  int h = w / 2, R = 2 * h;
  /* warped moving image on the (4h+1)^3 neighbourhood of j, which covers the
   * windows of every centre whose window holds j */
  int S = 2 * R + 1;
  double* mw = (double*)calloc((size_t)S * S * S, sizeof(double));
  double* ff = (double*)calloc((size_t)S * S * S, sizeof(double));
  unsigned char* in = (unsigned char*)calloc((size_t)S * S * S, 1);
  for (int dz = -R; dz <= R; dz++)
    for (int dy = -R; dy <= R; dy++)
      for (int dx = -R; dx <= R; dx++) {
        int zz = z + dz, yy = y + dy, xx = x + dx;
        long k = ((long)(dz + R) * S + (dy + R)) * S + (dx + R);
        if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx)
          continue;
        long i = IDX(zz, yy, xx);
        in[k] = 1;
        ff[k] = F[i];
        mw[k] = orc_sample(M, nz, ny, nx, xx + u[i], yy + u[N + i],
                           zz + u[2 * N + i], NULL);
      }
  double n = (double)w * w * w;
  long j = ((long)R * S + R) * S + R;
  double fj = ff[j], mj = mw[j], dS = 0.0;
  for (int cz = -h; cz <= h; cz++)
    for (int cy = -h; cy <= h; cy++)
      for (int cx = -h; cx <= h; cx++) {
        long kc = ((long)(cz + R) * S + (cy + R)) * S + (cx + R);
        if (!in[kc]) continue;
        double st[5] = {0, 0, 0, 0, 0};
        for (int dz = -h; dz <= h; dz++)
          for (int dy = -h; dy <= h; dy++)
            for (int dx = -h; dx <= h; dx++) {
              long k = ((long)(cz + dz + R) * S + (cy + dy + R)) * S +
                       (cx + dx + R);
              if (!in[k]) continue;
              st[0] += ff[k];
              st[1] += mw[k];
              st[2] += ff[k] * ff[k];
              st[3] += mw[k] * mw[k];
              st[4] += ff[k] * mw[k];
            }
        orc_local o = local_from_sums(st, w, eps);
        dS += o.alpha * (fj - o.muF) / n + o.beta * 2.0 * (mj - o.muM) / n;
      }
  long i = IDX(z, y, x);
  double d[3];
  orc_sample(M, nz, ny, nx, x + u[i], y + u[N + i], z + u[2 * N + i], d);
  for (int c = 0; c < 3; c++) g[c] = -dS * d[c];
  free(mw);
  free(ff);
  free(in);
}

double orc_cc_at(const double* F, const double* M, const double* u, int nz,
                 int ny, int nx, int w, double eps, int x, int y, int z) {
  long N = (long)nz * ny * nx;
  int h = w / 2;
  double st[5] = {0, 0, 0, 0, 0};
  for (int dz = -h; dz <= h; dz++)
    for (int dy = -h; dy <= h; dy++)
      for (int dx = -h; dx <= h; dx++) {
        int zz = z + dz, yy = y + dy, xx = x + dx;
        if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx)
          continue;
        long i = IDX(zz, yy, xx);
        double f = F[i];
        double m = orc_sample(M, nz, ny, nx, xx + u[i], yy + u[N + i],
                              zz + u[2 * N + i], NULL);
        st[0] += f;
        st[1] += m;
        st[2] += f * f;
        st[3] += m * m;
        st[4] += f * m;
      }
  return local_from_sums(st, w, eps).cc;
}

/* ------------------------------------------------------------------------ */
/* O4  Gaussian smoothing of the gradient (Eulerian descent, Sec. 2.1; the   */
/*     paper defers the filter to FireANTs).  Reading: taps k in [-R, R],    */
/*     R = ceil(3 sigma), weights exp(-k^2 / 2 sigma^2) normalised to sum 1, */
/*     zero outside the volume with no renormalisation at the border.        */
/* ------------------------------------------------------------------------ */

int orc_gauss_radius(double sigma) {
  if (!(sigma > 0.0)) return 0;
  return (int)ceil(3.0 * sigma - 1e-12);
}

void orc_gauss(const double* g, int nc, int nz, int ny, int nx, double sigma,
               double* out) {
  long N = (long)nz * ny * nx;
  int R = orc_gauss_radius(sigma);
  double* wt = (double*)malloc(sizeof(double) * (2 * R + 1));
  double tot = 0.0;
  for (int k = -R; k <= R; k++) {
    wt[k + R] = (R == 0) ? 1.0 : exp(-(double)k * k / (2.0 * sigma * sigma));
    tot += wt[k + R];
  }
  for (int k = 0; k <= 2 * R; k++) wt[k] /= tot;
  for (int c = 0; c < nc; c++) {
    const double* gc = g + c * N;
    double* oc = out + c * N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
      for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
          double s = 0.0;
          for (int dz = -R; dz <= R; dz++)
            for (int dy = -R; dy <= R; dy++)
              for (int dx = -R; dx <= R; dx++) {
                int zz = z + dz, yy = y + dy, xx = x + dx;
                if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 ||
                    xx >= nx)
                  continue;
                s += wt[dz + R] * wt[dy + R] * wt[dx + R] * gc[IDX(zz, yy, xx)];
              }
          oc[IDX(z, y, x)] = s;
        }
  }
  free(wt);
}

void orc_gauss_at(const double* g, int nc, int nz, int ny, int nx, double sigma,
                  int x, int y, int z, double* out) {
  long N = (long)nz * ny * nx;
  int R = orc_gauss_radius(sigma);
  double wt[64], tot = 0.0;
  for (int k = -R; k <= R; k++) {
    wt[k + R] = (R == 0) ? 1.0 : exp(-(double)k * k / (2.0 * sigma * sigma));
    tot += wt[k + R];
  }
  for (int k = 0; k <= 2 * R; k++) wt[k] /= tot;
  for (int c = 0; c < nc; c++) {
    double s = 0.0;
    for (int dz = -R; dz <= R; dz++)
      for (int dy = -R; dy <= R; dy++)
        for (int dx = -R; dx <= R; dx++) {
          int zz = z + dz, yy = y + dy, xx = x + dx;
          if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx)
            continue;
          s += wt[dz + R] * wt[dy + R] * wt[dx + R] * g[c * N + IDX(zz, yy, xx)];
        }
    out[c] = s;
  }
}

/* ------------------------------------------------------------------------ */
/* O5  Per-voxel rank-1 damped step (Sec. 2.2, eq. tile1; App. A).           */
/* ------------------------------------------------------------------------ */

void orc_closed_form(const double* gs, int nz, int ny, int nx, double r,
                     double lambda, double* du) {
  long N = (long)nz * ny * nx;
  for (long i = 0; i < N; i++) {
    double g0 = gs[i], g1 = gs[N + i], g2 = gs[2 * N + i];
    double den = g0 * g0 + g1 * g1 + g2 * g2 + lambda;
    du[i] = -r * g0 / den;
    du[N + i] = -r * g1 / den;
    du[2 * N + i] = -r * g2 / den;
  }
}

/* The linear system of App. A (eq. lm-local) solved without Sherman-Morrison:
 * Gaussian elimination with partial pivoting on the 3x3 matrix. */
void orc_explicit_solve(const double g[3], double r, double lambda,
                        double d[3]) {
  double A[3][4];
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 3; j++) A[i][j] = g[i] * g[j] + (i == j ? lambda : 0.0);
    A[i][3] = -r * g[i];
  }
  for (int k = 0; k < 3; k++) {
    int p = k;
    for (int i = k + 1; i < 3; i++)
      if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
    if (p != k)
      for (int j = 0; j < 4; j++) {
        double t = A[k][j];
        A[k][j] = A[p][j];
        A[p][j] = t;
      }
    for (int i = k + 1; i < 3; i++) {
      double f = A[i][k] / A[k][k];
      for (int j = k; j < 4; j++) A[i][j] -= f * A[k][j];
    }
  }
  for (int i = 2; i >= 0; i--) {
    double s = A[i][3];
    for (int j = i + 1; j < 3; j++) s -= A[i][j] * d[j];
    d[i] = s / A[i][i];
  }
}

/* ------------------------------------------------------------------------ */
/* Squared error and the Demons step (Sec. 2.2, the MSE needs no rewriting; */
/* Sec. 2.3, eq. demons).  Readings: the single scalar residual of the MSE  */
/* is r = sqrt(MSE), whose square is the loss (as 1 - LNCC is for LNCC),    */
/* and the gradient the step uses is N dr/du; the Demons step field is      */
/* Gaussian-smoothed with the gradient's sigma before eq. compositive.      */
/* ------------------------------------------------------------------------ */

double orc_mse_loss_grad(const double* F, const double* M, const double* u,
                         int nz, int ny, int nx, double* g_raw) {
  long N = (long)nz * ny * nx;
  double* Mw = (double*)malloc(sizeof(double) * N);
  double* dMw = (double*)malloc(sizeof(double) * 3 * N);
  orc_warp(M, u, nz, ny, nx, Mw, dMw);
  double s = 0.0;
  for (long i = 0; i < N; i++) s += (F[i] - Mw[i]) * (F[i] - Mw[i]);
  double L = s / (double)N;
  if (g_raw) {
    double r = sqrt(L);
    for (long i = 0; i < N; i++) {
      /* d r / d u_i = (1 / (2 r)) (2 / N) (Mw_i - F_i) dMw_i, times N */
      double c = r > 0.0 ? (Mw[i] - F[i]) / r : 0.0;
      for (int k = 0; k < 3; k++) g_raw[k * N + i] = c * dMw[k * N + i];
    }
  }
  free(Mw);
  free(dMw);
  return L;
}

void orc_demons_step(const double* F, const double* M, const double* u, int nz,
                     int ny, int nx, double lambda, double* du) {
  long N = (long)nz * ny * nx;
  double* Mw = (double*)malloc(sizeof(double) * N);
  double* n = (double*)malloc(sizeof(double) * 3 * N);
  orc_warp(M, u, nz, ny, nx, Mw, n);
  for (long i = 0; i < N; i++) {
    double r = F[i] - Mw[i];
    double a = n[i], b = n[N + i], c = n[2 * N + i];
    double den = a * a + b * b + c * c + lambda;
    du[i] = r * a / den;
    du[N + i] = r * b / den;
    du[2 * N + i] = r * c / den;
  }
  free(Mw);
  free(n);
}

/* ------------------------------------------------------------------------ */
/* Mutual information (Sec. 2.2: (log2 B - MI)^2).  Readings: cubic B-spline */
/* Parzen windows for both images (a partition of unity, so the fixed       */
/* marginal does not depend on u); each image mapped to bin coordinates     */
/* 1 + (B - 3)(v - lo)/(hi - lo) over its range (the moving range extended  */
/* to 0, the value outside the volume), keeping every window inside the B   */
/* bins; MI in bits; r = log2 B - MI and the step uses N dr/du.             */
/* ------------------------------------------------------------------------ */

double orc_bspline3(double t) {
  double a = fabs(t);
  if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
  if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
  return 0.0;
}

double orc_dbspline3(double t) {
  double a = fabs(t), s = t < 0.0 ? -1.0 : 1.0;
  if (a < 1.0) return s * (-2.0 * a + 1.5 * a * a);
  if (a < 2.0) return -s * 0.5 * (2.0 - a) * (2.0 - a);
  return 0.0;
}

static void range_of(const double* v, long n, int with_zero, double* lo, double* hi) {
  double a = v[0], b = v[0];
  for (long i = 1; i < n; i++) {
    if (v[i] < a) a = v[i];
    if (v[i] > b) b = v[i];
  }
  if (with_zero) {
    if (a > 0.0) a = 0.0;
    if (b < 0.0) b = 0.0;
  }
  if (!(b > a)) b = a + 1.0;
  *lo = a;
  *hi = b;
}

double orc_mi_loss_grad(const double* F, const double* M, const double* u, int nz,
                        int ny, int nx, int B, double* g_raw, double* hist) {
  long N = (long)nz * ny * nx;
  double flo, fhi, mlo, mhi;
  range_of(F, N, 0, &flo, &fhi);
  range_of(M, N, 1, &mlo, &mhi);
  double sf = (B - 3) / (fhi - flo), sm = (B - 3) / (mhi - mlo);
  double* Mw = (double*)malloc(sizeof(double) * N);
  double* dMw = (double*)malloc(sizeof(double) * 3 * N);
  double* p = (double*)calloc((size_t)B * B, sizeof(double));
  orc_warp(M, u, nz, ny, nx, Mw, dMw);
  for (long i = 0; i < N; i++) {
    double fh = 1.0 + (F[i] - flo) * sf, mh = 1.0 + (Mw[i] - mlo) * sm;
    for (int a = 0; a < B; a++) {
      double wa = orc_bspline3(fh - a);
      if (wa == 0.0) continue;
      for (int b = 0; b < B; b++) p[a * B + b] += wa * orc_bspline3(mh - b);
    }
  }
  for (int k = 0; k < B * B; k++) p[k] /= (double)N;
  double* pa = (double*)calloc(B, sizeof(double));
  double* pb = (double*)calloc(B, sizeof(double));
  for (int a = 0; a < B; a++)
    for (int b = 0; b < B; b++) {
      pa[a] += p[a * B + b];
      pb[b] += p[a * B + b];
    }
  double mi = 0.0;
  for (int a = 0; a < B; a++)
    for (int b = 0; b < B; b++)
      if (p[a * B + b] > 0.0) mi += p[a * B + b] * log2(p[a * B + b] / (pa[a] * pb[b]));
  if (g_raw) {
    for (long i = 0; i < N; i++) {
      double fh = 1.0 + (F[i] - flo) * sf, mh = 1.0 + (Mw[i] - mlo) * sm;
      double dmi = 0.0; /* d MI / d Mw_i, times N */
      for (int a = 0; a < B; a++) {
        double wa = orc_bspline3(fh - a);
        if (wa == 0.0) continue;
        for (int b = 0; b < B; b++) {
          double pab = p[a * B + b];
          if (pab <= 0.0) continue;
          dmi += wa * orc_dbspline3(mh - b) * sm * log2(pab / pb[b]);
        }
      }
      for (int k = 0; k < 3; k++) g_raw[k * N + i] = -dmi * dMw[k * N + i];
    }
  }
  if (hist) memcpy(hist, p, sizeof(double) * B * B);
  free(Mw);
  free(dMw);
  free(p);
  free(pa);
  free(pb);
  return -mi;
}

/* The loss (and with g_raw the gradient the step uses) of the similarity. */
static double sim_loss_grad(const orc_params* p, const double* F, const double* M,
                            const double* u, int nz, int ny, int nx, double* g_raw) {
  if (p->similarity == 0)
    return orc_loss_grad(F, M, u, nz, ny, nx, p->window, p->cc_eps, g_raw);
  if (p->similarity == 3) return orc_mi_loss_grad(F, M, u, nz, ny, nx, p->mi_bins, g_raw, NULL);
  return orc_mse_loss_grad(F, M, u, nz, ny, nx, g_raw);
}

/* The residual whose square is the minimised loss (Sec. 2.2). */
static double residual(const orc_params* p, double L) {
  if (p->similarity == 0) return 1.0 + L;
  if (p->similarity == 3) return log2((double)p->mi_bins) + L;
  return sqrt(L > 0.0 ? L : 0.0);
}

/* ------------------------------------------------------------------------ */
/* O5' Pooled Hessian over tiles of side k (Sec. 2.2, eq. tilen; Sec. 3.2).  */
/*   Readings: the tiles are the disjoint k^3 blocks of the grid from the    */
/*   origin (the ablation sweeps even sides too, so not a centred window);   */
/*   a block cut by a far face keeps its voxels inside the volume; the       */
/*   pooled matrix is the mean of the voxels' rank-1 products, so that k = 1 */
/*   is eq. tile1 and lambda keeps its scale for every k; each voxel solves  */
/*   with its own smoothed gradient on the right-hand side.                  */
/* ------------------------------------------------------------------------ */

void orc_tile_hessian(const double* gs, int nz, int ny, int nx, int k, double* H) {
  long N = (long)nz * ny * nx;
  int tx = (nx + k - 1) / k, ty = (ny + k - 1) / k, tz = (nz + k - 1) / k;
  for (int bz = 0; bz < tz; bz++)
    for (int by = 0; by < ty; by++)
      for (int bx = 0; bx < tx; bx++) {
        double h[6] = {0, 0, 0, 0, 0, 0};
        long cnt = 0;
        for (int z = bz * k; z < bz * k + k && z < nz; z++)
          for (int y = by * k; y < by * k + k && y < ny; y++)
            for (int x = bx * k; x < bx * k + k && x < nx; x++) {
              long i = IDX(z, y, x);
              double a = gs[i], b = gs[N + i], c = gs[2 * N + i];
              h[0] += a * a;
              h[1] += b * b;
              h[2] += c * c;
              h[3] += a * b;
              h[4] += a * c;
              h[5] += b * c;
              cnt++;
            }
        double* o = H + 6 * (((long)bz * ty + by) * tx + bx);
        for (int e = 0; e < 6; e++) o[e] = h[e] / (double)cnt;
      }
}

/* Gaussian elimination with partial pivoting of A d = b (3x3). */
static void solve3(double A[3][4], double d[3]) {
  for (int k = 0; k < 3; k++) {
    int p = k;
    for (int i = k + 1; i < 3; i++)
      if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
    if (p != k)
      for (int j = 0; j < 4; j++) {
        double t = A[k][j];
        A[k][j] = A[p][j];
        A[p][j] = t;
      }
    for (int i = k + 1; i < 3; i++) {
      double f = A[i][k] / A[k][k];
      for (int j = k; j < 4; j++) A[i][j] -= f * A[k][j];
    }
  }
  for (int i = 2; i >= 0; i--) {
    double s = A[i][3];
    for (int j = i + 1; j < 3; j++) s -= A[i][j] * d[j];
    d[i] = s / A[i][i];
  }
}

void orc_tile_step(const double* gs, int nz, int ny, int nx, int k, double r,
                   double lambda, double* du) {
  long N = (long)nz * ny * nx;
  int tx = (nx + k - 1) / k, ty = (ny + k - 1) / k, tz = (nz + k - 1) / k;
  double* H = (double*)malloc(sizeof(double) * 6 * (size_t)tx * ty * tz);
  orc_tile_hessian(gs, nz, ny, nx, k, H);
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        long i = IDX(z, y, x);
        const double* h = H + 6 * (((long)(z / k) * ty + y / k) * tx + x / k);
        double A[3][4] = {{h[0] + lambda, h[3], h[4], -r * gs[i]},
                          {h[3], h[1] + lambda, h[5], -r * gs[N + i]},
                          {h[4], h[5], h[2] + lambda, -r * gs[2 * N + i]}};
        double d[3];
        solve3(A, d);
        du[i] = d[0];
        du[N + i] = d[1];
        du[2 * N + i] = d[2];
      }
  free(H);
}

/* ------------------------------------------------------------------------ */
/* Adam comparator (the paper's baseline, Sec. 3 and Sec. 3.5).  Readings:   */
/*   the moments are taken of the smoothed gradient (the gradient the LM    */
/*   step uses: Eulerian descent smooths the gradient before the optimizer  */
/*   acts on it); the bias-corrected step -lr mhat / (sqrt(vhat) + eps) is  */
/*   integrated by eq. compositive like the LM step; every step is kept.    */
/* ------------------------------------------------------------------------ */

void orc_adam_direction(const double* gs, double* m, double* v, long n, long t,
                        const orc_adam_params* a, double* du) {
  double c1 = 1.0 - pow(a->beta1, (double)t), c2 = 1.0 - pow(a->beta2, (double)t);
  for (long i = 0; i < n; i++) {
    m[i] = a->beta1 * m[i] + (1.0 - a->beta1) * gs[i];
    v[i] = a->beta2 * v[i] + (1.0 - a->beta2) * gs[i] * gs[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    du[i] = -a->lr * mh / (sqrt(vh) + a->eps);
  }
}

/* ------------------------------------------------------------------------ */
/* O6  Integration (Sec. 2.1, eq. compositive).  Reading: v = Delta u with   */
/*     no further normalisation; u is resampled with the O1 conventions.     */
/* ------------------------------------------------------------------------ */

void orc_integrate(const double* u, const double* v, int nz, int ny, int nx,
                   double eps, int compositive, double* unew) {
  long N = (long)nz * ny * nx;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        long i = IDX(z, y, x);
        double ev0 = eps * v[i], ev1 = eps * v[N + i], ev2 = eps * v[2 * N + i];
        for (int c = 0; c < 3; c++) {
          double ev = c == 0 ? ev0 : (c == 1 ? ev1 : ev2);
          double base;
          if (compositive)
            base = orc_sample(u + c * N, nz, ny, nx, x + ev0, y + ev1, z + ev2,
                              NULL);
          else
            base = u[c * N + i];
          unew[c * N + i] = ev + base;
        }
      }
}

/* ------------------------------------------------------------------------ */
/* O7  Decision: damping rule (eq. lambda-update) and rejection              */
/*     (eq. rejection, Sec. 3.4).                                            */
/*   Readings: with fewer than two accepted losses the reference term        */
/*   |L^(t-1) - L^(t-2)| is 0; a non-finite loss is always rejected; on      */
/*   rejection lambda <- min(mu+ lambda, lambda_max); after max_retries      */
/*   consecutive rejections with lambda at lambda_max the pair is frozen.    */
/* ------------------------------------------------------------------------ */

static double clampd(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

int orc_decide(const orc_params* p, orc_state* s, double cand_loss, int force) {
  s->cand_loss = cand_loss;
  if (s->stalled) {
    s->accepted = 0;
    return 0;
  }
  int acc;
  if (force >= 0)
    acc = force ? 1 : 0;
  else if (!isfinite(cand_loss))
    acc = 0;
  else if (p->tau < 0.0)
    acc = 1;
  else {
    double ref = s->n_hist >= 2 ? fabs(s->loss - s->loss_prev) : 0.0;
    acc = !((cand_loss - s->loss) > p->tau * ref);
  }
  if (acc) {
    double f = (cand_loss > s->loss) ? p->lambda_inc : p->lambda_dec;
    s->lambda = clampd(f * s->lambda, p->lambda_min, p->lambda_max);
    s->loss_prev = s->loss;
    s->loss = cand_loss;
    s->n_hist += 1;
    s->retries = 0;
  } else {
    s->lambda = clampd(p->lambda_inc * s->lambda, p->lambda_min, p->lambda_max);
    s->retries += 1;
    if (s->retries >= p->max_retries && s->lambda >= p->lambda_max)
      s->stalled = 1;
  }
  s->accepted = acc;
  return acc;
}

/* ------------------------------------------------------------------------ */
/* One pair: begin (evaluate the starting field) and one LM attempt.         */
/* ------------------------------------------------------------------------ */

void orc_begin(const orc_params* p, const double* F, const double* M,
               const double* u, int nz, int ny, int nx, double lambda0,
               orc_state* s, double* gs_out) {
  long N = (long)nz * ny * nx;
  double* g = (double*)malloc(sizeof(double) * 3 * N);
  double L = sim_loss_grad(p, F, M, u, nz, ny, nx, g);
  orc_gauss(g, 3, nz, ny, nx, p->grad_sigma, gs_out);
  free(g);
  s->lambda = lambda0;
  s->loss = L;
  s->loss_prev = L;
  s->cand_loss = L;
  s->n_hist = 1;
  s->retries = 0;
  s->accepted = 1;
  s->stalled = 0;
}

int orc_attempt(const orc_params* p, const double* F, const double* M,
                double* u, double* gs, int nz, int ny, int nx, orc_state* s,
                int force) {
  if (s->stalled) {
    s->accepted = 0;
    return 0;
  }
  long N = (long)nz * ny * nx;
  double r = residual(p, s->loss); /* e.g. 1 - LNCC of the accepted field */
  double* v = (double*)malloc(sizeof(double) * 3 * N);
  double* ut = (double*)malloc(sizeof(double) * 3 * N);
  double* g = (double*)malloc(sizeof(double) * 3 * N);
  if (p->similarity == 2) {
    /* Demons: the per-voxel step of the accepted field, smoothed */
    orc_demons_step(F, M, u, nz, ny, nx, s->lambda, g);
    orc_gauss(g, 3, nz, ny, nx, p->grad_sigma, v);
  } else if (p->tile > 1) {
    orc_tile_step(gs, nz, ny, nx, p->tile, r, s->lambda, v);
  } else {
    orc_closed_form(gs, nz, ny, nx, r, s->lambda, v);
  }
  orc_integrate(u, v, nz, ny, nx, p->step_eps, p->compositive, ut);
  double Lc = sim_loss_grad(p, F, M, ut, nz, ny, nx, g);
  int acc = orc_decide(p, s, Lc, force);
  if (acc) {
    memcpy(u, ut, sizeof(double) * 3 * N);
    orc_gauss(g, 3, nz, ny, nx, p->grad_sigma, gs);
  }
  free(v);
  free(ut);
  free(g);
  return acc;
}

void orc_adam_iter(const orc_params* p, const orc_adam_params* a, const double* F,
                   const double* M, double* u, double* gs, double* m, double* v,
                   int nz, int ny, int nx, long t, orc_state* s) {
  long N = (long)nz * ny * nx;
  double* du = (double*)malloc(sizeof(double) * 3 * N);
  double* ut = (double*)malloc(sizeof(double) * 3 * N);
  double* g = (double*)malloc(sizeof(double) * 3 * N);
  orc_adam_direction(gs, m, v, 3 * N, t, a, du);
  orc_integrate(u, du, nz, ny, nx, p->step_eps, p->compositive, ut);
  double L = sim_loss_grad(p, F, M, ut, nz, ny, nx, g);
  orc_gauss(g, 3, nz, ny, nx, p->grad_sigma, gs);
  memcpy(u, ut, sizeof(double) * 3 * N);
  s->loss_prev = s->loss;
  s->loss = L;
  s->cand_loss = L;
  s->n_hist += 1;
  s->accepted = 1;
  free(du);
  free(ut);
  free(g);
}

/* ------------------------------------------------------------------------ */
/* O8  Pyramid (Sec. 2.1: coarse-to-fine, each level inherits the warp).     */
/*   Readings: images are average-pooled; the field is upsampled x2 with     */
/*   voxel-centre alignment (fine index i maps to coarse (i - 0.5)/2,        */
/*   clamped to the coarse grid) and its values are doubled.                 */
/* ------------------------------------------------------------------------ */

void orc_avgpool(const double* a, int nz, int ny, int nx, int f, double* out) {
  int cz = nz / f, cy = ny / f, cx = nx / f;
  double inv = 1.0 / ((double)f * f * f);
  for (int z = 0; z < cz; z++)
    for (int y = 0; y < cy; y++)
      for (int x = 0; x < cx; x++) {
        double s = 0.0;
        for (int k = 0; k < f; k++)
          for (int j = 0; j < f; j++)
            for (int i = 0; i < f; i++)
              s += a[IDX(z * f + k, y * f + j, x * f + i)];
        out[((long)z * cy + y) * cx + x] = s * inv;
      }
}

static void src_coord(int i, int nc, long* i0, long* i1, double* t) {
  double s = (i - 0.5) / 2.0;
  if (s < 0.0) s = 0.0;
  if (s > nc - 1) s = nc - 1;
  double b = floor(s);
  *i0 = (long)b;
  *i1 = *i0 + 1 < nc ? *i0 + 1 : *i0;
  *t = s - b;
}

void orc_upsample_field(const double* uc, int nzc, int nyc, int nxc,
                        double* uf, int nz, int ny, int nx) {
  long Nc = (long)nzc * nyc * nxc, N = (long)nz * ny * nx;
  for (int c = 0; c < 3; c++)
    for (int z = 0; z < nz; z++)
      for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
          long z0, z1, y0, y1, x0, x1;
          double tz, ty, tx;
          src_coord(z, nzc, &z0, &z1, &tz);
          src_coord(y, nyc, &y0, &y1, &ty);
          src_coord(x, nxc, &x0, &x1, &tx);
          const double* a = uc + c * Nc;
#define C(zz, yy, xx) a[((zz) * nyc + (yy)) * nxc + (xx)]
          double v = (1 - tz) * ((1 - ty) * ((1 - tx) * C(z0, y0, x0) + tx * C(z0, y0, x1)) +
                                 ty * ((1 - tx) * C(z0, y1, x0) + tx * C(z0, y1, x1))) +
                     tz * ((1 - ty) * ((1 - tx) * C(z1, y0, x0) + tx * C(z1, y0, x1)) +
                           ty * ((1 - tx) * C(z1, y1, x0) + tx * C(z1, y1, x1)));
#undef C
          uf[c * N + IDX(z, y, x)] = 2.0 * v;
        }
}

/* ------------------------------------------------------------------------ */
/* O9  Folded voxels: det(I + grad u) <= 0.  Central differences inside,     */
/*     one-sided first-order differences on the faces.                       */
/* ------------------------------------------------------------------------ */

static double dcomp(const double* a, int nz, int ny, int nx, int z, int y,
                    int x, int axis) {
  int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
  int i = axis == 0 ? x : (axis == 1 ? y : z);
  if (n < 2) return 0.0;
  int lo = i > 0 ? i - 1 : i, hi = i < n - 1 ? i + 1 : i;
  double vlo, vhi;
  if (axis == 0) {
    vlo = a[IDX(z, y, lo)];
    vhi = a[IDX(z, y, hi)];
  } else if (axis == 1) {
    vlo = a[IDX(z, lo, x)];
    vhi = a[IDX(z, hi, x)];
  } else {
    vlo = a[IDX(lo, y, x)];
    vhi = a[IDX(hi, y, x)];
  }
  return (vhi - vlo) / (double)(hi - lo);
}

long orc_folded_count(const double* u, int nz, int ny, int nx, double* det) {
  long N = (long)nz * ny * nx, count = 0;
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        double J[3][3];
        for (int c = 0; c < 3; c++)
          for (int d = 0; d < 3; d++)
            J[c][d] = (c == d ? 1.0 : 0.0) + dcomp(u + c * N, nz, ny, nx, z, y, x, d);
        double D = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                   J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                   J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (det) det[IDX(z, y, x)] = D;
        if (D <= 0.0) count++;
      }
  return count;
}
