// Internal declarations shared by the HIP kernels and the C-ABI layer of
// liblmreg.  Not installed; the public interface is include/lmreg.h.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
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
  double adam_pow1;  // beta1^t and beta2^t of the next Adam step t (its bias
  double adam_pow2;  // corrections are 1 - beta^t)
};

// Scalars of the decision rule (eq. lambda-update, eq. rejection).
struct DecideParams {
  double lambda_inc, lambda_dec, lambda_min, lambda_max, tau;
  int max_retries;
  double adam_beta1, adam_beta2;  // for the bias corrections kept in the state
  int similarity;                 // lmr_similarity: how the residual r follows from L
  int mi_bins;                    // B of the mutual information
};

// The scalar residual of the least-squares form of the loss (Sec. 2.2):
// r = 1 - LNCC = 1 + L for LNCC (L = -LNCC), r = log2 B - MI = log2 B + L
// for mutual information (L = -MI), r = sqrt(MSE) for the squared error
// (its square is the loss).
__host__ __device__ inline double residual_of(double L, int similarity, int bins) {
  if (similarity == LMR_SIM_LNCC) return 1.0 + L;
  if (similarity == LMR_SIM_MI) return log2(static_cast<double>(bins)) + L;
  return sqrt(L > 0.0 ? L : 0.0);
}



// Direction of the update besides eq. tile1 (lmr_params.tile, .optimizer).
struct StepExtra {
  int mode;                 // 0 eq. tile1, 1 eq. tilen (pooled Hessian), 2 Adam,
                            // 3 a given direction (the smoothed Demons step, in G)
  const double* H;          // mode 1: mean g g^T per tile [tiles][6]
  int k, tx, ty;            // mode 1: tile side, tiles along x and y
  float* m;                 // mode 2: moments [3][N] each
  float* v;
  float b1, ob1, b2, ob2;   // mode 2: decays and 1 - decays
  float lr, aeps;           // mode 2: step length, epsilon
};

struct Geom {
  int nz, ny, nx;
  long long N;
};

// ---------------------------------------------------------------- helpers
// Voxel counts are below 2^31 (checked at context creation), so indices
// within one channel are 32-bit.
__device__ __forceinline__ float ldf(const float* p, int i) { return p[i]; }
__device__ __forceinline__ float ldf(const uint16_t* p, int i) {
  return __uint_as_float(static_cast<uint32_t>(p[i]) << 16);
}

// Integer cell and fractional offset of the sample coordinate base + d, as
// if base + d were formed exactly: floor(base + d) = base + floor(d) for an
// integer base, and d - floor(d) is exact in FP32, so the choice of cell does
// not depend on the rounding of a float sum.  Offsets beyond +-1e9 (and NaN)
// are clamped far outside the volume.
__device__ __forceinline__ void cell(int base, float d, int& i0, float& f) {
  const float dc = fminf(fmaxf(d, -1e9f), 1e9f);
  const float fl = floorf(dc);
  i0 = base + static_cast<int>(fl);
  f = dc - fl;
}

// The trilinear cell of the point (x+dx, y+dy, z+dz): lower corner, weights
// and whether all eight corners lie inside the volume.
struct Cell {
  int x0, y0, z0;
  float fx, fy, fz;
  bool interior;
  int base;  // linear index of the lower corner (meaningful when interior)
};

__device__ __forceinline__ Cell make_cell(const Geom& g, int x, int y, int z, float dx,
                                          float dy, float dz) {
  Cell c;
  cell(x, dx, c.x0, c.fx);
  cell(y, dy, c.y0, c.fy);
  cell(z, dz, c.z0, c.fz);
  c.interior = (unsigned)c.x0 < (unsigned)(g.nx - 1) &&
               (unsigned)c.y0 < (unsigned)(g.ny - 1) &&
               (unsigned)c.z0 < (unsigned)(g.nz - 1);
  c.base = c.interior ? (c.z0 * g.ny + c.y0) * g.nx + c.x0 : 0;
  return c;
}

// The eight corner values v[4k + 2j + i] (i along x, j along y, k along z);
// corners outside the volume read as 0.
template <typename T>
__device__ __forceinline__ void corners(const T* __restrict__ V, const Geom& g,
                                        const Cell& c, float v[8]) {
  if (c.interior) {
    const int b = c.base, sy = g.nx, sz = g.nx * g.ny;
    v[0] = ldf(V, b);
    v[1] = ldf(V, b + 1);
    v[2] = ldf(V, b + sy);
    v[3] = ldf(V, b + sy + 1);
    v[4] = ldf(V, b + sz);
    v[5] = ldf(V, b + sz + 1);
    v[6] = ldf(V, b + sz + sy);
    v[7] = ldf(V, b + sz + sy + 1);
    return;
  }
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int xi = c.x0 + i, yi = c.y0 + j, zi = c.z0 + k;
        const bool in = (unsigned)xi < (unsigned)g.nx && (unsigned)yi < (unsigned)g.ny &&
                        (unsigned)zi < (unsigned)g.nz;
        v[4 * k + 2 * j + i] = in ? ldf(V, (zi * g.ny + yi) * g.nx + xi) : 0.0f;
      }
}

// Interpolated value from the corners; grad (may be null) receives the
// derivative of the interpolant on the cell.
// Each weighted pair a*x + b*y is one product and one fused multiply-add.
__device__ __forceinline__ float lerp2(float a, float x, float b, float y) {
  return fmaf(b, y, a * x);
}
__device__ __forceinline__ float interp(const Cell& c, const float v[8], float* grad) {
  const float gx0 = 1.0f - c.fx, gy0 = 1.0f - c.fy, gz0 = 1.0f - c.fz;
  const float c00 = lerp2(gx0, v[0], c.fx, v[1]);
  const float c01 = lerp2(gx0, v[2], c.fx, v[3]);
  const float c10 = lerp2(gx0, v[4], c.fx, v[5]);
  const float c11 = lerp2(gx0, v[6], c.fx, v[7]);
  const float c0 = lerp2(gy0, c00, c.fy, c01);
  const float c1 = lerp2(gy0, c10, c.fy, c11);
  if (grad) {
    const float d00 = v[1] - v[0], d01 = v[3] - v[2];
    const float d10 = v[5] - v[4], d11 = v[7] - v[6];
    grad[0] = lerp2(gz0, lerp2(gy0, d00, c.fy, d01), c.fz, lerp2(gy0, d10, c.fy, d11));
    grad[1] = lerp2(gz0, c01 - c00, c.fz, c11 - c10);
    grad[2] = c1 - c0;
  }
  return lerp2(gz0, c0, c.fz, c1);
}

// Trilinear sample of V at (x+dx, y+dy, z+dz) with zero padding.
template <typename T>
__device__ __forceinline__ float trilinear(const T* __restrict__ V, const Geom& g,
                                           int x, int y, int z, float dx, float dy,
                                           float dz, float* grad) {
  const Cell c = make_cell(g, x, y, z, dx, dy, dz);
  float v[8];
  corners(V, g, c, v);
  return interp(c, v, grad);
}

// ------------------------------------------------------- buffer resources
// A buffer resource addresses one channel with a 32-bit byte offset; the
// hardware checks the offset against the channel size and returns 0 for any
// read beyond it (a write beyond it is dropped), so out-of-volume reads need
// no branch and can never fault.  Channels hold fewer than 2^30 voxels.
constexpr int kBufDword3 = 0x00020000;  // raw 32-bit access on gfx9-class GPUs
constexpr unsigned kFarOffset = 0xFFFFFFF0u;  // always beyond num_records
// element index whose 4-byte offset lies beyond any channel (< 2^30 voxels)
constexpr unsigned kFarIndex = 0x3FFFFFFFu;

struct RBuf {
  __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ RBuf make_rbuf(const void* p, unsigned bytes) {
  return RBuf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                                (int)bytes, kBufDword3)};
}
template <typename T>
__device__ __forceinline__ RBuf make_rbuf_n(const T* p, int n) {
  return make_rbuf(p, static_cast<unsigned>(n) * sizeof(T));
}

// element i of a buffer holding T (float or BF16 bits), as float
__device__ __forceinline__ float bload(const RBuf& b, unsigned i, float) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(b.r, i * 4u, 0, 0));
}
__device__ __forceinline__ float bload(const RBuf& b, unsigned i, uint16_t) {
  const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(b.r, i * 2u, 0, 0);
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}
template <typename T>
__device__ __forceinline__ float bld(const RBuf& b, unsigned i) {
  return bload(b, i, T());
}
// byte-offset form: o is already a byte offset (kFarOffset reads 0)
__device__ __forceinline__ float bld_off(const RBuf& b, unsigned o, float) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(b.r, o, 0, 0));
}
__device__ __forceinline__ void bst(const RBuf& b, unsigned i, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), b.r, i * 4u, 0, 0);
}

// The trilinear cell addressed through buffers.  Each corner coordinate is
// clamped into the volume, so all loads are in range and issued
// unconditionally; zero padding is applied through the weights instead: the
// weight (and derivative sign) of a corner plane outside the volume is 0.
// This gives the same sums, rounding included, as interpolating corners
// replaced by 0.  (Offsets are never formed by wrap-around: adjacent loads
// may be fused into one wider access, which the hardware range-checks as a
// whole.)
//
// A gather costs the address and data paths of the vector memory unit per
// load instruction and lane, not per byte, so for FP32 volumes the two
// corners of a row are read with one 8-byte load at x = clamp(x0, 0, nx-2):
// corner x0 is its second element only when x0 = nx-1, corner x0+1 its first
// only when x0 = -1 (any other out-of-row corner has weight 0).
struct BCell {
  unsigned r[4];            // element offset of the corner rows (j, k) at r[2k + j]
  unsigned xa, xb;          // clamped x of corners 0 and 1
  unsigned xc;              // start of the two-element row read (nx >= 2)
  bool hi0, lo1;            // corner 0 from the pair's 2nd element, corner 1 from its 1st
  float wx0, wx1, wy0, wy1, wz0, wz1;  // 1-f, f per axis; 0 outside
  float sx0, sx1, sy0, sy1, sz0, sz1;  // -1, +1 per axis; 0 outside
};

__device__ __forceinline__ BCell make_bcell(const Geom& g, int x, int y, int z, float dx,
                                            float dy, float dz) {
  int x0, y0, z0;
  float fx, fy, fz;
  cell(x, dx, x0, fx);
  cell(y, dy, y0, fy);
  cell(z, dz, z0, fz);
  const bool x0i = (unsigned)x0 < (unsigned)g.nx, x1i = (unsigned)(x0 + 1) < (unsigned)g.nx;
  const bool y0i = (unsigned)y0 < (unsigned)g.ny, y1i = (unsigned)(y0 + 1) < (unsigned)g.ny;
  const bool z0i = (unsigned)z0 < (unsigned)g.nz, z1i = (unsigned)(z0 + 1) < (unsigned)g.nz;
  BCell c;
  c.wx0 = x0i ? 1.0f - fx : 0.0f;
  c.wx1 = x1i ? fx : 0.0f;
  c.wy0 = y0i ? 1.0f - fy : 0.0f;
  c.wy1 = y1i ? fy : 0.0f;
  c.wz0 = z0i ? 1.0f - fz : 0.0f;
  c.wz1 = z1i ? fz : 0.0f;
  c.sx0 = x0i ? -1.0f : 0.0f;
  c.sx1 = x1i ? 1.0f : 0.0f;
  c.sy0 = y0i ? -1.0f : 0.0f;
  c.sy1 = y1i ? 1.0f : 0.0f;
  c.sz0 = z0i ? -1.0f : 0.0f;
  c.sz1 = z1i ? 1.0f : 0.0f;
  c.xa = min(max(x0, 0), g.nx - 1);
  c.xb = min(max(x0 + 1, 0), g.nx - 1);
  c.xc = min(max(x0, 0), max(g.nx - 2, 0));
  c.hi0 = x0 >= g.nx - 1;
  c.lo1 = x0 < 0;
  const int ya = min(max(y0, 0), g.ny - 1), yb = min(max(y0 + 1, 0), g.ny - 1);
  const int za = min(max(z0, 0), g.nz - 1), zb = min(max(z0 + 1, 0), g.nz - 1);
  c.r[0] = (za * g.ny + ya) * g.nx;
  c.r[1] = (za * g.ny + yb) * g.nx;
  c.r[2] = (zb * g.ny + ya) * g.nx;
  c.r[3] = (zb * g.ny + yb) * g.nx;
  return c;
}

// Corner values v[4k + 2j + i] (i along x, j along y, k along z).
template <typename T>
__device__ __forceinline__ void bcorners(const RBuf& b, const Geom&, const BCell& c,
                                         float v[8]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[2 * q] = bld<T>(b, c.r[q] + c.xa);
    v[2 * q + 1] = bld<T>(b, c.r[q] + c.xb);
  }
}
// BF16 volumes with an even row length of at least 4: the two corners of a
// row come from one 8-byte load of four elements starting at the even
// index min(xc & ~1, nx - 4) (4-byte aligned, never past the row end), which
// holds both clamped corners xa and xb.
template <>
__device__ __forceinline__ void bcorners<uint16_t>(const RBuf& b, const Geom& g,
                                                   const BCell& c, float v[8]) {
  if ((g.nx & 1) || g.nx < 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[2 * q] = bld<uint16_t>(b, c.r[q] + c.xa);
      v[2 * q + 1] = bld<uint16_t>(b, c.r[q] + c.xb);
    }
    return;
  }
  const unsigned base = min(c.xc & ~1u, static_cast<unsigned>(g.nx - 4));
  const unsigned sa = 16u * (c.xa - base), sb = 16u * (c.xb - base);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const auto p = __builtin_amdgcn_raw_buffer_load_b64(b.r, (c.r[q] + base) * 2u, 0, 0);
    const unsigned long long w =
        (static_cast<unsigned long long>(p[1]) << 32) | static_cast<unsigned long long>(p[0]);
    v[2 * q] = __uint_as_float(static_cast<uint32_t>((w >> sa) & 0xFFFFu) << 16);
    v[2 * q + 1] = __uint_as_float(static_cast<uint32_t>((w >> sb) & 0xFFFFu) << 16);
  }
}
template <>
__device__ __forceinline__ void bcorners<float>(const RBuf& b, const Geom& g, const BCell& c,
                                                float v[8]) {
  if (g.nx < 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[2 * q] = v[2 * q + 1] = bld<float>(b, c.r[q] + c.xa);
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const auto p = __builtin_amdgcn_raw_buffer_load_b64(b.r, (c.r[q] + c.xc) * 4u, 0, 0);
    const float lo = __uint_as_float(p[0]), hi = __uint_as_float(p[1]);
    v[2 * q] = c.hi0 ? hi : lo;
    v[2 * q + 1] = c.lo1 ? lo : hi;
  }
}

// Interpolated value; grad (may be null) receives the derivative of the
// interpolant on the cell along x, y, z.
__device__ __forceinline__ float binterp(const BCell& c, const float v[8], float* grad) {
  const float c00 = lerp2(c.wx0, v[0], c.wx1, v[1]);
  const float c01 = lerp2(c.wx0, v[2], c.wx1, v[3]);
  const float c10 = lerp2(c.wx0, v[4], c.wx1, v[5]);
  const float c11 = lerp2(c.wx0, v[6], c.wx1, v[7]);
  const float c0 = lerp2(c.wy0, c00, c.wy1, c01);
  const float c1 = lerp2(c.wy0, c10, c.wy1, c11);
  if (grad) {
    const float d00 = lerp2(c.sx0, v[0], c.sx1, v[1]);
    const float d01 = lerp2(c.sx0, v[2], c.sx1, v[3]);
    const float d10 = lerp2(c.sx0, v[4], c.sx1, v[5]);
    const float d11 = lerp2(c.sx0, v[6], c.sx1, v[7]);
    grad[0] = lerp2(c.wz0, lerp2(c.wy0, d00, c.wy1, d01), c.wz1,
                    lerp2(c.wy0, d10, c.wy1, d11));
    grad[1] = lerp2(c.wz0, lerp2(c.sy0, c00, c.sy1, c01), c.wz1,
                    lerp2(c.sy0, c10, c.sy1, c11));
    grad[2] = lerp2(c.sz0, c0, c.sz1, c1);
  }
  return lerp2(c.wz0, c0, c.wz1, c1);
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

// The forward pass's block count (one cc partial per block); launch_fwd
// checks its launch against it.
int fwd_num_blocks(const Geom& g, const lmr_params& p);
// compute units of the current device (cached per device; 256 when the query
// fails)
int device_cus();
int gauss_radius(double sigma);

hipError_t launch_warp(const void* M, lmr_dtype t, const float* u, const Geom& g,
                       float* Mw, float* dMw, hipStream_t s);
// P1: closed form + compositive integration + warp of M at the candidate.
// Explicit mode (st == null): reads u_in, g_smooth, r, lambda, writes u_out.
// In state mode dMw (may be null) receives the derivative of the warped image
// at the candidate, for P4.
hipError_t launch_update(const void* M, lmr_dtype t, const Geom& g,
                         const lmr_params& p, const DevState* st,
                         const float* G, float* U0, float* U1, const float* u_in,
                         float* u_out, double r, double lambda, float* Mw, float* dMw,
                         hipStream_t s, const StepExtra* extra = nullptr);
// Mutual information (k_mi.hip).  Histogram blocks of the forward pass:
// kMiBlocks at most (mi_hist_blocks(N)); their partial histograms take
// kMiBlocks * bins^2 unsigned 64-bit counts.
constexpr int kMiBlocks = 256;
int mi_hist_blocks(long long N);
// map[0..3] = (lo_F, s_F, lo_M, s_M) of the bin coordinates, from the
// ranges of F and M (part: 4 * kMiBlocks floats of scratch).
hipError_t launch_mi_range(const void* F, const void* M, lmr_dtype t, const Geom& g, int bins,
                           float* part, double* map, hipStream_t s);
// Joint histogram of F and Mw, p (FP64 [bins^2]), the gradient table tab
// (FP64 [bins^2]) and partials[0] = N MI; a frozen pair is skipped.
hipError_t launch_mi_fwd(const void* F, lmr_dtype t, const float* Mw, const Geom& g, int bins,
                         const double* map, unsigned long long* hpart, double* p, double* tab,
                         double* partials, const DevState* st, hipStream_t s);
// g = N dr/du from tab (only after an acceptance with a state); dMw may
// alias graw.
hipError_t launch_mi_bwd(const void* F, lmr_dtype t, const float* Mw, const float* dMw,
                         const Geom& g, int bins, const double* map, const double* tab,
                         const DevState* st, float* graw, hipStream_t s);
// Squared-error similarity (k_mse.hip).  mse_fwd: one FP64 partial of
// -sum (F - Mw)^2 per block, nparts blocks (sq_map, may be null: the squared
// errors); a frozen pair is skipped.  mse_bwd: g = (Mw - F) dMw / r with r
// the state's residual (only after an acceptance) or sqrt(*loss) without a
// state; dMw may alias graw.
hipError_t launch_mse_fwd(const void* F, lmr_dtype t, const float* Mw, const Geom& g,
                          int nparts, double* partials, float* sq_map, const DevState* st,
                          hipStream_t s);
hipError_t launch_mse_bwd(const void* F, lmr_dtype t, const float* Mw, const float* dMw,
                          const Geom& g, const DevState* st, const double* loss, float* graw,
                          hipStream_t s);
// Demons step (eq. demons): du = r_x n_x / (|n_x|^2 + lambda) from keep =
// [r_x | n_x] ([4][N]) of the accepted field; keep is refreshed by
// demons_keep after an acceptance (always without a state).
hipError_t launch_demons_force(const float* keep, const Geom& g, const DevState* st,
                               float* du, hipStream_t s);
hipError_t launch_demons_keep(const void* F, lmr_dtype t, const float* Mw, const float* dMw,
                              const Geom& g, const DevState* st, float* keep,
                              hipStream_t s);
// Mean of g g^T over every tile of side k (eq. tilen) into H [tiles][6];
// need = 2 with a state: only after an acceptance (the gradient changed).
hipError_t launch_tile_hessian(const float* G, const Geom& g, int k, double* H,
                               const DevState* st, int need, hipStream_t s);

// Window mean and variance of F (FP64, [2][N]), read by every P2 on that F.
hipError_t launch_fstat(const void* F, lmr_dtype t, const Geom& g, const lmr_params& p,
                        double* fstat, hipStream_t s);
// P2: LNCC forward; writes adjoint maps, per-block partials and optionally cc.
// fstat: launch_fstat's output for the same F.
// nparts: fwd_num_blocks(g, p), the partials' length (hipErrorInvalidValue if
// the launch would differ, e.g. on a device with another CU count).
hipError_t launch_fwd(const void* F, lmr_dtype t, const float* Mw, const double* fstat,
                      const Geom& g, const lmr_params& p, const DevState* st, float* maps,
                      double* partials, int nparts, float* cc_map, hipStream_t s);
// P3: FP64 reduction of the partials and the decision.
// mode 0: attempt (force -1/0/1), mode 1: begin (lambda0), mode 2: probe.
hipError_t launch_decide(DevState* st, const double* partials, int nparts,
                         long long N, const DecideParams& dp, int mode, int force,
                         double lambda0, double* probe, hipStream_t s);
// P4: LNCC backward and warp backward -> raw gradient.  The field is U[cur]
// in state mode, u_explicit otherwise.  dMw (may be null, may alias graw):
// the derivative of M at x + u(x) stored by P1 for the accepted candidate;
// null gathers it from M.
hipError_t launch_bwd(const void* F, const void* M, lmr_dtype t, const float* Mw,
                      const float* maps, const Geom& g, const lmr_params& p,
                      const DevState* st, const float* U0, const float* U1,
                      const float* u_explicit, const float* dMw, float* graw,
                      hipStream_t s);
// P5: Gaussian smoothing of the raw gradient.
hipError_t launch_smooth(const float* graw, const Geom& g, const lmr_params& p,
                         const DevState* st, float* out, hipStream_t s);
hipError_t launch_avgpool(const void* in, lmr_dtype t, int nz, int ny, int nx, int f,
                          float* out, hipStream_t s);
hipError_t launch_upsample_field(const float* uc, int nzc, int nyc, int nxc, float* uf,
                                 hipStream_t s);
// *count = number of voxels with det(I + grad u) <= 0; det (may be null)
// receives the determinant map.
hipError_t launch_folds(const float* u, const Geom& g, unsigned long long* count,
                        float* det, hipStream_t s);
// Overwrite every field of *st except `cur` with the fields of v.
hipError_t launch_set_state(DevState* st, const DevState& v, hipStream_t s);
// dst[0..n) = v (a kernel, so that graph captures hold no memset node).
hipError_t launch_fill(float* dst, long long n, float v, hipStream_t s);
// Copy U[cur] (state mode) into dst.
hipError_t launch_copy_cur(const DevState* st, const float* U0, const float* U1,
                           float* dst, long long n, hipStream_t s);

}  // namespace lmr
