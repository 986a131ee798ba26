// Per-voxel kernels of one LM attempt and the on-device decision.
//
//   k_warp    Mw(x) = M(x + u(x))                       (Sec. 1, eq. 1)
//   k_update  du = -r g/(|g|^2 + lambda)                (Sec. 2.2, eq. tile1)
//             u~ = eps du + u o (Id + eps du)           (Sec. 2.1, eq. compositive)
//             Mw = M o (Id + u~)  (the candidate's warped image, fused here)
//   k_decide  FP64 loss reduction, damping rule and rejection test
//             (Sec. 2.2, eq. lambda-update / eq. delta-loss; Sec. 3.4, eq. rejection)
#include "decide.h"
#include "lmr_internal.h"
#include "update.h"

#include <math.h>

#include <algorithm>

namespace lmr {

namespace {

constexpr int kBX = 64, kBY = 4;
constexpr int kUpdZ = 1;  // voxels per thread (along z) of the update kernel (measured: 1 or 2
                          // best; 4 loses occupancy)

__device__ __forceinline__ bool voxel(const Geom& g, int& x, int& y, int& z, int& i) {
  x = blockIdx.x * kBX + threadIdx.x;
  y = blockIdx.y * kBY + threadIdx.y;
  z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return false;
  i = (z * g.ny + y) * g.nx + x;
  return true;
}

template <typename T>
__global__ void __launch_bounds__(kBX* kBY)
    k_warp(const T* __restrict__ M, const float* __restrict__ u, Geom g,
           float* __restrict__ Mw, float* __restrict__ dMw) {
  int x, y, z, i;
  if (!voxel(g, x, y, z, i)) return;
  const int N = static_cast<int>(g.N);
  const RBuf bm = make_rbuf_n(M, N);
  const BCell c = make_bcell(g, x, y, z, u[i], u[N + i], u[2 * N + i]);
  float v[8], d[3];
  bcorners<T>(bm, g, c, v);
  Mw[i] = binterp(c, v, dMw ? d : nullptr);
  if (dMw) {
    dMw[i] = d[0];
    dMw[N + i] = d[1];
    dMw[2 * N + i] = d[2];
  }
}

template <typename T>
__global__ void __launch_bounds__(kBX* kBY)
    k_update(const T* __restrict__ M, Geom g, const DevState* __restrict__ st,
             const float* __restrict__ G, float* U0, float* U1,
             const float* u_in, float* u_out, float r_arg, float lam_arg,
             float eps, int compositive, float* __restrict__ Mw, float* dMw) {
  UpdateArgs a;
  if (st) {
    if (st->stalled) return;
    a = update_args_from_state(st, U0, U1, G, Mw, eps, compositive);
    a.dMw = dMw;
  } else {
    a.uin = u_in;
    a.uo = u_out;
    a.G = G;
    a.Mw = Mw;
    a.dMw = nullptr;
    a.r = r_arg;
    a.lam = lam_arg;
    a.eps = eps;
    a.compositive = compositive;
  }
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  if (x >= g.nx || y >= g.ny) return;
  update_voxels<T, kUpdZ>(M, g, a, x, y, blockIdx.z * kUpdZ);
}

// The same attempt step with the accepted field staged in LDS.  A block owns
// a 32 x 8 column of voxels and marches along z through a chunk of planes,
// keeping the planes z-1, z, z+1 of the three field channels (with a
// one-voxel halo in x and y) in a ring of LDS slots.  The compositive
// gather u(x + eps du) reads its eight corners from LDS whenever every
// component of eps du lies in [-1, 1) (the cell's corners are then within one
// voxel of x), and from memory otherwise.  The staged values are the field's
// own, and out-of-volume corners carry weight 0 either way, so each voxel's
// result is that of update_voxel (up to the sign of an exact zero).
constexpr int kSX = 32, kSY = 8, kSNT = kSX * kSY;
constexpr int kSLX = kSX + 2, kSLY = kSY + 2, kSPOS = kSLX * kSLY;
constexpr int kSPER = (kSPOS + kSNT - 1) / kSNT;
constexpr int kSlots = 4;  // planes z-1..z+1 in use while z+2 is written
constexpr int kStagedMinBlocks = 1024, kStagedBlocks = 1024;

template <typename T>
__global__ void __launch_bounds__(kSNT)
    k_update_staged(const T* __restrict__ M, Geom g, const DevState* __restrict__ st,
                    const float* __restrict__ G, float* U0, float* U1, const float* u_in,
                    float* u_out, float r_arg, float lam_arg, float eps,
                    float* __restrict__ Mw, float* dMw, int cz) {
  UpdateArgs a;
  if (st) {
    if (st->stalled) return;
    a = update_args_from_state(st, U0, U1, G, Mw, eps, 1);
    a.dMw = dMw;
  } else {
    a.uin = u_in;
    a.uo = u_out;
    a.G = G;
    a.Mw = Mw;
    a.dMw = nullptr;
    a.r = r_arg;
    a.lam = lam_arg;
    a.eps = eps;
    a.compositive = 1;
  }
  __shared__ float s_u[kSlots][3][kSLY][kSLX];
  const int N = static_cast<int>(g.N), plane = g.nx * g.ny;
  const int lx = threadIdx.x % kSX, ly = threadIdx.x / kSX;
  // one-dimensional grid; each XCD receives a contiguous range of tiles
  // (x fastest, then y, then z-chunk) and shares their halos in its L2
  const int tiles_x = (g.nx + kSX - 1) / kSX, tiles_y = (g.ny + kSY - 1) / kSY;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = (tile % tiles_x) * kSX, by = ((tile / tiles_x) % tiles_y) * kSY;
  const int z0 = (tile / (tiles_x * tiles_y)) * cz, z1 = min(z0 + cz, g.nz);
  const int x = bx + lx, y = by + ly;
  const bool own = x < g.nx && y < g.ny;
  const RBuf bu[3] = {make_rbuf_n(a.uin, N), make_rbuf_n(a.uin + N, N),
                      make_rbuf_n(a.uin + 2 * N, N)};

  // staged positions of this thread (padding positions read 0)
  int pidx[kSPER];
  bool pin[kSPER];
#pragma unroll
  for (int p = 0; p < kSPER; ++p) {
    const int i = threadIdx.x + p * kSNT;
    const int yy = i / kSLX, xx = i - yy * kSLX;
    const int gy = by - 1 + yy, gx = bx - 1 + xx;
    pin[p] = i < kSPOS && (unsigned)gy < (unsigned)g.ny && (unsigned)gx < (unsigned)g.nx;
    pidx[p] = pin[p] ? gy * g.nx + gx : 0;
  }
  float pre[kSPER][3];
  auto fetch = [&](int zi) {
    const bool zin = (unsigned)zi < (unsigned)g.nz;
#pragma unroll
    for (int p = 0; p < kSPER; ++p) {
      const unsigned o = (zin && pin[p]) ? static_cast<unsigned>(zi * plane + pidx[p])
                                         : kFarIndex;
#pragma unroll
      for (int c = 0; c < 3; ++c) pre[p][c] = bld<float>(bu[c], o);
    }
  };
  auto slot = [](int zi) { return (zi + kSlots) % kSlots; };  // zi >= -1
  auto commit = [&](int zi) {
    const int sl = slot(zi);
#pragma unroll
    for (int p = 0; p < kSPER; ++p) {
      const int i = threadIdx.x + p * kSNT;
      if (i < kSPOS) {
        const int yy = i / kSLX, xx = i - yy * kSLX;
#pragma unroll
        for (int c = 0; c < 3; ++c) s_u[sl][c][yy][xx] = pre[p][c];
      }
    }
  };

  fetch(z0 - 1);
  commit(z0 - 1);
  fetch(z0);
  commit(z0);
  fetch(z0 + 1);
  const RBuf bm = make_rbuf_n(M, N);
  const RBuf bg[3] = {make_rbuf_n(a.G, N), make_rbuf_n(a.G + N, N),
                      make_rbuf_n(a.G + 2 * N, N)};
  // the gradient of the next plane is in flight while a plane is processed
  const unsigned col = own ? static_cast<unsigned>(y * g.nx + x) : kFarIndex;
  float gn[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    gn[c] = bld<float>(bg[c], own ? static_cast<unsigned>(z0 * plane) + col : kFarIndex);
  // The image gather M(x + u~) of a plane stays in flight while the next
  // plane's field work runs; it is finished (interpolated and stored) then.
  const bool warp = M && a.Mw;
  BCell pc;
  float pv[8];
  int pi = -1;  // voxel of the pending image gather (-1: none)
  auto finish = [&]() {
    if (pi < 0) return;
    float d[3];
    a.Mw[pi] = binterp(pc, pv, a.dMw ? d : nullptr);
    if (a.dMw) {
      a.dMw[pi] = d[0];
      a.dMw[N + pi] = d[1];
      a.dMw[2 * N + pi] = d[2];
    }
  };
  for (int z = z0; z < z1; ++z) {
    // slot(z+1) last held plane z-3, whose readers finished before the
    // barrier of the previous iteration
    commit(z + 1);
    if (z + 2 <= z1) fetch(z + 2);
    const float g0 = gn[0], g1 = gn[1], g2 = gn[2];
    if (z + 1 < z1) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        gn[c] = bld<float>(bg[c], own ? static_cast<unsigned>((z + 1) * plane) + col
                                      : kFarIndex);
    }
    __syncthreads();
    if (!own) continue;
    const int i = (z * g.ny + y) * g.nx + x;
    const float s = -a.r / fmaf(g2, g2, fmaf(g1, g1, fmaf(g0, g0, a.lam)));
    const float e0 = a.eps * (s * g0), e1 = a.eps * (s * g1), e2 = a.eps * (s * g2);
    const BCell c = make_bcell(g, x, y, z, e0, e1, e2);
    float b[3];
    if (e0 >= -1.0f && e0 < 1.0f && e1 >= -1.0f && e1 < 1.0f && e2 >= -1.0f && e2 < 1.0f) {
      // lower corner (x + floor(e0), y + floor(e1), z + floor(e2)), each
      // floor in {-1, 0}: staged column lx + floor + 1, row ly + floor + 1
      const int cx = lx + 1 + (e0 < 0.0f ? -1 : 0);
      const int cy = ly + 1 + (e1 < 0.0f ? -1 : 0);
      const int cz0 = z + (e2 < 0.0f ? -1 : 0);
      const int s0 = slot(cz0), s1 = slot(cz0 + 1);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float v[8];
        v[0] = s_u[s0][ch][cy][cx];
        v[1] = s_u[s0][ch][cy][cx + 1];
        v[2] = s_u[s0][ch][cy + 1][cx];
        v[3] = s_u[s0][ch][cy + 1][cx + 1];
        v[4] = s_u[s1][ch][cy][cx];
        v[5] = s_u[s1][ch][cy][cx + 1];
        v[6] = s_u[s1][ch][cy + 1][cx];
        v[7] = s_u[s1][ch][cy + 1][cx + 1];
        b[ch] = binterp(c, v, nullptr);
      }
    } else {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float v[8];
        bcorners<float>(bu[ch], g, c, v);
        b[ch] = binterp(c, v, nullptr);
      }
    }
    const float n0 = e0 + b[0], n1 = e1 + b[1], n2 = e2 + b[2];
    a.uo[i] = n0;
    a.uo[N + i] = n1;
    a.uo[2 * N + i] = n2;
    finish();
    if (warp) {
      pc = make_bcell(g, x, y, z, n0, n1, n2);
      bcorners<T>(bm, g, pc, pv);
      pi = i;
    }
  }
  if (own) finish();
}

constexpr int kDecideThreads = 256;

__global__ void __launch_bounds__(kDecideThreads)
    k_decide(DevState* st, const double* __restrict__ partials, int nparts,
             long long N, DecideParams dp, int mode, int force, double lambda0,
             double* probe) {
  decide_block<kDecideThreads>(st, partials, nparts, N, dp, mode, force, lambda0, probe);
}

__global__ void k_copy_cur(const DevState* __restrict__ st, const float* U0,
                           const float* U1, float* __restrict__ dst, long long n) {
  const float* src = st->cur ? U1 : U0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_fill(float* __restrict__ dst, long long n, float v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = v;
}

__global__ void k_set_state(DevState* st, DevState v) {
  v.cur = st->cur;
  *st = v;
}

dim3 vox_grid(const Geom& g) {
  return dim3((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY, g.nz);
}

unsigned flat_grid(long long n) {
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  return static_cast<unsigned>(blocks);
}

}  // namespace

hipError_t launch_warp(const void* M, lmr_dtype t, const float* u, const Geom& g,
                       float* Mw, float* dMw, hipStream_t s) {
  dim3 blk(kBX, kBY);
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_warp<uint16_t>, vox_grid(g), blk, 0, s,
                       static_cast<const uint16_t*>(M), u, g, Mw, dMw);
  else
    hipLaunchKernelGGL(k_warp<float>, vox_grid(g), blk, 0, s,
                       static_cast<const float*>(M), u, g, Mw, dMw);
  return hipGetLastError();
}

hipError_t launch_update(const void* M, lmr_dtype t, const Geom& g,
                         const lmr_params& p, const DevState* st, const float* G,
                         float* U0, float* U1, const float* u_in, float* u_out,
                         double r, double lambda, float* Mw, float* dMw, hipStream_t s) {
  dim3 blk(kBX, kBY);
  const float rf = static_cast<float>(r), lf = static_cast<float>(lambda);
  const float eps = static_cast<float>(p.step_eps);
  if (p.compositive) {
    // staged form when the volume gives enough z-chunks of at least 8 planes
    // (small pyramid levels are latency-bound and keep one plane per block)
    const int cols = ((g.nx + kSX - 1) / kSX) * ((g.ny + kSY - 1) / kSY);
    if ((long long)cols * (g.nz / 8) >= kStagedMinBlocks) {
      int cz = (int)(((long long)g.nz * cols + kStagedBlocks - 1) / kStagedBlocks);
      cz = std::max(cz, 8);
      const dim3 sgrid(cols * ((g.nz + cz - 1) / cz));
      if (t == LMR_BF16)
        hipLaunchKernelGGL(k_update_staged<uint16_t>, sgrid, dim3(kSNT), 0, s,
                           static_cast<const uint16_t*>(M), g, st, G, U0, U1, u_in, u_out,
                           rf, lf, eps, Mw, dMw, cz);
      else
        hipLaunchKernelGGL(k_update_staged<float>, sgrid, dim3(kSNT), 0, s,
                           static_cast<const float*>(M), g, st, G, U0, U1, u_in, u_out, rf,
                           lf, eps, Mw, dMw, cz);
      return hipGetLastError();
    }
  }
  const dim3 grid((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY, (g.nz + kUpdZ - 1) / kUpdZ);
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_update<uint16_t>, grid, blk, 0, s,
                       static_cast<const uint16_t*>(M), g, st, G, U0, U1, u_in, u_out,
                       rf, lf, eps, p.compositive, Mw, dMw);
  else
    hipLaunchKernelGGL(k_update<float>, grid, blk, 0, s,
                       static_cast<const float*>(M), g, st, G, U0, U1, u_in, u_out, rf,
                       lf, eps, p.compositive, Mw, dMw);
  return hipGetLastError();
}

hipError_t launch_decide(DevState* st, const double* partials, int nparts,
                         long long N, const DecideParams& dp, int mode, int force,
                         double lambda0, double* probe, hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(kDecideThreads), 0, s, st, partials,
                     nparts, N, dp, mode, force, lambda0, probe);
  return hipGetLastError();
}

hipError_t launch_copy_cur(const DevState* st, const float* U0, const float* U1,
                           float* dst, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_cur, dim3(flat_grid(n)), dim3(256), 0, s, st, U0, U1, dst,
                     n);
  return hipGetLastError();
}

hipError_t launch_set_state(DevState* st, const DevState& v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, s, st, v);
  return hipGetLastError();
}

hipError_t launch_fill(float* dst, long long n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(flat_grid(n)), dim3(256), 0, s, dst, n, v);
  return hipGetLastError();
}

}  // namespace lmr
