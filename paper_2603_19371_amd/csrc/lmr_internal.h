// Internal declarations shared by the HIP kernels and the C-ABI layer of
// liblmreg.  Not installed; the public interface is include/lmreg.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lmreg.h"

namespace lmr {

// Device-resident optimizer state of one pair.  Every kernel of an attempt
// reads it at entry, so a sequence of attempts needs no host round trip.
struct DevState {
  double lambda;     // damping of the next attempt
  double loss;       // L of the accepted field
  double loss_prev;  // L of the field accepted before it
  double cand_loss;  // L of the last candidate
  double r;          // residual 1 - LNCC = 1 + loss of the accepted field
  int32_t n_hist;
  int32_t retries;
  int32_t accepted;  // decision of the last attempt
  int32_t stalled;
  int32_t cur;       // index (0/1) of the field buffer holding the accepted field
  int32_t pad_;
  int64_t attempts;
};

// Scalars of the decision rule (eq. lambda-update, eq. rejection).
struct DecideParams {
  double lambda_inc, lambda_dec, lambda_min, lambda_max, tau;
  int max_retries;
};

struct Geom {
  int nz, ny, nx;
  long long N;
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ float ldf(const float* p, long long i) { return p[i]; }
__device__ __forceinline__ float ldf(const uint16_t* p, long long i) {
  return __uint_as_float(static_cast<uint32_t>(p[i]) << 16);
}

// Integer cell and fractional offset of the sample coordinate base + d.
// base + d is formed in FP64, which is exact for an FP32 d and an integer
// base, so the choice of cell does not depend on the rounding of a float sum.
__device__ __forceinline__ void cell(int base, float d, int& i0, float& f) {
  double p = static_cast<double>(base) + static_cast<double>(d);
  double fl = floor(p);
  i0 = static_cast<int>(fl);
  f = static_cast<float>(p - fl);
}

// Trilinear sample of V at (x+dx, y+dy, z+dz) with zero padding; when grad
// is non-null it receives the derivative of the interpolant on the cell.
template <typename T>
__device__ __forceinline__ float trilinear(const T* __restrict__ V, const Geom g,
                                           int x, int y, int z, float dx, float dy,
                                           float dz, float* grad) {
  int x0, y0, z0;
  float fx, fy, fz;
  cell(x, dx, x0, fx);
  cell(y, dy, y0, fy);
  cell(z, dz, z0, fz);
  float c[2][2][2];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        int xi = x0 + i, yi = y0 + j, zi = z0 + k;
        bool in = (unsigned)xi < (unsigned)g.nx && (unsigned)yi < (unsigned)g.ny &&
                  (unsigned)zi < (unsigned)g.nz;
        c[k][j][i] = in ? ldf(V, ((long long)zi * g.ny + yi) * g.nx + xi) : 0.0f;
      }
  float gx0 = 1.0f - fx, gy0 = 1.0f - fy, gz0 = 1.0f - fz;
  // interpolate along x first
  float c00 = gx0 * c[0][0][0] + fx * c[0][0][1];
  float c01 = gx0 * c[0][1][0] + fx * c[0][1][1];
  float c10 = gx0 * c[1][0][0] + fx * c[1][0][1];
  float c11 = gx0 * c[1][1][0] + fx * c[1][1][1];
  float c0 = gy0 * c00 + fy * c01;
  float c1 = gy0 * c10 + fy * c11;
  if (grad) {
    float d00 = c[0][0][1] - c[0][0][0], d01 = c[0][1][1] - c[0][1][0];
    float d10 = c[1][0][1] - c[1][0][0], d11 = c[1][1][1] - c[1][1][0];
    grad[0] = gz0 * (gy0 * d00 + fy * d01) + fz * (gy0 * d10 + fy * d11);
    grad[1] = gz0 * (c01 - c00) + fz * (c11 - c10);
    grad[2] = c1 - c0;
  }
  return gz0 * c0 + fz * c1;
}

// Bijective remap of a linear block index so that the blocks which the
// dispatcher sends to one XCD (block id modulo 8) receive a contiguous range
// of tiles and share their halos in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  constexpr int kXcd = 8;
  int per = nb / kXcd, rem = nb % kXcd;
  int x = b % kXcd, k = b / kXcd;
  return (x < rem) ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// ---------------------------------------------------------------- launchers
// All return hipSuccess or the launch error.  `st` may be null (explicit mode).
struct StepBuffers {
  float* U[2];      // field ping-pong, [3][N] each
  float* G;         // smoothed gradient of the accepted field, [3][N]
  float* graw;      // raw gradient, [3][N]
  float* maps;      // LNCC adjoint maps alpha, alpha mu_F, beta, beta mu_M, [4][N]
  float* Mw;        // warped moving image, [N]
  double* partials; // one FP64 partial sum of cc per forward block
  int nparts;
  DevState* st;
  double* probe;    // scalar loss written by the probe reduction
};

int fwd_num_blocks(const Geom& g, int window);
int gauss_radius(double sigma);

hipError_t launch_warp(const void* M, lmr_dtype t, const float* u, const Geom& g,
                       float* Mw, float* dMw, hipStream_t s);
// P1: closed form + compositive integration + warp of M at the candidate.
// Explicit mode (st == null): reads u_in, g_smooth, r, lambda, writes u_out.
hipError_t launch_update(const void* M, lmr_dtype t, const Geom& g,
                         const lmr_params& p, const DevState* st,
                         const float* G, float* U0, float* U1, const float* u_in,
                         float* u_out, double r, double lambda, float* Mw,
                         hipStream_t s);
// P2: LNCC forward; writes adjoint maps, per-block partials and optionally cc.
hipError_t launch_fwd(const void* F, lmr_dtype t, const float* Mw, const Geom& g,
                      const lmr_params& p, const DevState* st, float* maps,
                      double* partials, float* cc_map, hipStream_t s);
// P3: FP64 reduction of the partials and the decision.
// mode 0: attempt (force -1/0/1), mode 1: begin (lambda0), mode 2: probe.
hipError_t launch_decide(DevState* st, const double* partials, int nparts,
                         long long N, const DecideParams& dp, int mode, int force,
                         double lambda0, double* probe, hipStream_t s);
// P4: LNCC backward and warp backward -> raw gradient.  The field is U[cur]
// in state mode, u_explicit otherwise.
hipError_t launch_bwd(const void* F, const void* M, lmr_dtype t, const float* Mw,
                      const float* maps, const Geom& g, const lmr_params& p,
                      const DevState* st, const float* U0, const float* U1,
                      const float* u_explicit, float* graw, hipStream_t s);
// P5: Gaussian smoothing of the raw gradient.
hipError_t launch_smooth(const float* graw, const Geom& g, const lmr_params& p,
                         const DevState* st, float* out, hipStream_t s);
// Overwrite every field of *st except `cur` with the fields of v.
hipError_t launch_set_state(DevState* st, const DevState& v, hipStream_t s);
// dst[0..n) = v (a kernel, so that graph captures hold no memset node).
hipError_t launch_fill(float* dst, long long n, float v, hipStream_t s);
// Copy U[cur] (state mode) into dst.
hipError_t launch_copy_cur(const DevState* st, const float* U0, const float* U1,
                           float* dst, long long n, hipStream_t s);

}  // namespace lmr
