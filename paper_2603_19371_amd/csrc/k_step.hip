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
#include <atomic>

namespace lmr {

namespace {

constexpr int kBX = 64, kBY = 4;
constexpr int kUpdZ = 1;  // voxels per thread (along z) of the update kernel (measured: 2
                          // is 11 % slower at 80x96x112, 4 loses occupancy)

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

// The step policy of mode MODE (0 eq. tile1, 1 eq. tilen, 2 Adam, 3 a given
// direction field: the smoothed Demons step) for the
// update arguments a; r and lambda in FP64 (state or explicit arguments).
template <int MODE>
struct StepOf;
template <>
struct StepOf<0> {
  using type = PointStep;
  __device__ static PointStep make(const UpdateArgs& a, const Geom& g, const StepExtra&,
                                   const DevState*, double, double) {
    return point_step(a, g);
  }
};
template <>
struct StepOf<1> {
  using type = TileStep;
  __device__ static TileStep make(const UpdateArgs& a, const Geom& g, const StepExtra& x,
                                  const DevState*, double r, double lam) {
    return TileStep{a.G, x.H, static_cast<int>(g.N), x.k, x.tx, x.ty, r, lam, a.eps};
  }
};
template <>
struct StepOf<2> {
  using type = AdamStep;
  __device__ static AdamStep make(const UpdateArgs& a, const Geom& g, const StepExtra& x,
                                  const DevState* st, double, double) {
    return AdamStep{a.G,
                    x.m,
                    x.v,
                    static_cast<int>(g.N),
                    x.b1,
                    x.ob1,
                    x.b2,
                    x.ob2,
                    static_cast<float>(1.0 - st->adam_pow1),
                    static_cast<float>(1.0 - st->adam_pow2),
                    x.lr,
                    x.aeps,
                    a.eps};
  }
};

template <>
struct StepOf<3> {
  using type = GivenStep;
  __device__ static GivenStep make(const UpdateArgs& a, const Geom& g, const StepExtra&,
                                   const DevState*, double, double) {
    return GivenStep{a.G, static_cast<int>(g.N), a.eps};
  }
};

template <typename T, int MODE>
__global__ void __launch_bounds__(kBX* kBY)
    k_update(const T* __restrict__ M, Geom g, const DevState* __restrict__ st,
             const float* __restrict__ G, float* U0, float* U1,
             const float* u_in, float* u_out, double r_arg, double lam_arg,
             float eps, int compositive, float* __restrict__ Mw, float* dMw, StepExtra ex) {
  UpdateArgs a;
  double r = r_arg, lam = lam_arg;
  if (st) {
    if (st->stalled) return;
    a = update_args_from_state(st, U0, U1, G, Mw, eps, compositive);
    a.dMw = dMw;
    r = st->r;
    lam = st->lambda;
  } else {
    a.uin = u_in;
    a.uo = u_out;
    a.G = G;
    a.Mw = Mw;
    a.dMw = nullptr;
    a.r = static_cast<float>(r_arg);
    a.lam = static_cast<float>(lam_arg);
    a.eps = eps;
    a.compositive = compositive;
  }
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  if (x >= g.nx || y >= g.ny) return;
  const auto step = StepOf<MODE>::make(a, g, ex, st, r, lam);
  update_voxels<T, kUpdZ>(M, g, a, step, x, y, blockIdx.z * kUpdZ);
}

// The update with the accepted field staged in LDS (staged_update_tile),
// one tile per block.
constexpr int kStagedMinBlocks = 1024, kStagedBlocks = 1024;

template <typename T, int MODE>
__global__ void __launch_bounds__(kSNT)
    k_update_staged(const T* __restrict__ M, Geom g, const DevState* __restrict__ st,
                    const float* __restrict__ G, float* U0, float* U1, const float* u_in,
                    float* u_out, double r_arg, double lam_arg, float eps,
                    float* __restrict__ Mw, float* dMw, int cz, StepExtra ex) {
  UpdateArgs a;
  double r = r_arg, lam = lam_arg;
  if (st) {
    if (st->stalled) return;
    a = update_args_from_state(st, U0, U1, G, Mw, eps, 1);
    a.dMw = dMw;
    r = st->r;
    lam = st->lambda;
  } else {
    a.uin = u_in;
    a.uo = u_out;
    a.G = G;
    a.Mw = Mw;
    a.dMw = nullptr;
    a.r = static_cast<float>(r_arg);
    a.lam = static_cast<float>(lam_arg);
    a.eps = eps;
    a.compositive = 1;
  }
  // one-dimensional grid; each XCD receives a contiguous range of tiles
  // (x fastest, then y, then z-chunk) and shares their halos in its L2
  const int tiles_x = (g.nx + kSX - 1) / kSX, tiles_y = (g.ny + kSY - 1) / kSY;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = (tile % tiles_x) * kSX, by = ((tile / tiles_x) % tiles_y) * kSY;
  const int z0 = (tile / (tiles_x * tiles_y)) * cz, z1 = min(z0 + cz, g.nz);
  staged_update_tile(M, g, a, StepOf<MODE>::make(a, g, ex, st, r, lam), bx, by, z0, z1);
}

// Mean of g g^T over each tile of side k, accumulated in FP64 in the order
// z, y, x of the tile's voxels; one thread per tile.
__global__ void __launch_bounds__(256)
    k_tile_hessian(const float* __restrict__ G, Geom g, int k, int tx, int ty, int ntiles,
                   double* __restrict__ H, const DevState* __restrict__ st, int need) {
  if (st && need) {
    if (st->stalled) return;
    if (need == 2 && !st->accepted) return;
  }
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  const int N = static_cast<int>(g.N);
  const int bx = t % tx, by = (t / tx) % ty, bz = t / (tx * ty);
  double h[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int cnt = 0;
  for (int z = bz * k; z < min(bz * k + k, g.nz); ++z)
    for (int y = by * k; y < min(by * k + k, g.ny); ++y)
      for (int x = bx * k; x < min(bx * k + k, g.nx); ++x) {
        const int i = (z * g.ny + y) * g.nx + x;
        const double a = G[i], b = G[N + i], c = G[2 * N + i];
        h[0] += a * a;
        h[1] += b * b;
        h[2] += c * c;
        h[3] += a * b;
        h[4] += a * c;
        h[5] += b * c;
        ++cnt;
      }
#pragma unroll
  for (int e = 0; e < 6; ++e) H[6LL * t + e] = h[e] / cnt;
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

// compute units of the current device, cached per device (a tiling
// heuristic only: 256 when the query fails)
int device_cus() {
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cus[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int n = 0;
    const bool ok =
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess;
    v = ok && n > 0 ? n : 256;
    cus[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

namespace {

// z-chunk of the staged form.  The blocks of a launch are co-resident and
// each marches its chunk plane by plane, so a launch lasts about (most blocks
// on one CU) x (planes per chunk + the two halo planes).  Among the chunk
// counts that give chunks of at least 8 planes and at least 3/4 of
// kStagedBlocks blocks, take the one that minimises that product (fewer
// blocks on a tie).
int staged_cz(int cols, int nz) {
  const long long cus = device_cus();
  int best_cz = 0;
  long long best = 0;
  for (int n = 1; n <= nz / 8; ++n) {
    const int cz = (nz + n - 1) / n;
    const long long blocks = (long long)cols * ((nz + cz - 1) / cz);
    if (blocks < kStagedBlocks * 3 / 4) continue;
    const long long cost = ((blocks + cus - 1) / cus) * (cz + 2);
    if (best_cz == 0 || cost < best) {
      best = cost;
      best_cz = cz;
    }
  }
  if (best_cz == 0)
    best_cz = std::max(8, (int)(((long long)nz * cols + kStagedBlocks - 1) / kStagedBlocks));
  return best_cz;
}

}  // namespace

namespace {

template <int MODE>
hipError_t update_mode(const void* M, lmr_dtype t, const Geom& g, const lmr_params& p,
                       const DevState* st, const float* G, float* U0, float* U1,
                       const float* u_in, float* u_out, double r, double lambda, float* Mw,
                       float* dMw, hipStream_t s, const StepExtra& ex) {
  dim3 blk(kBX, kBY);
  const float eps = static_cast<float>(p.step_eps);
  if (p.compositive) {
    // staged form when the volume gives enough z-chunks of at least 8 planes
    // (small pyramid levels are latency-bound and keep one plane per block)
    const int cols = ((g.nx + kSX - 1) / kSX) * ((g.ny + kSY - 1) / kSY);
    if ((long long)cols * (g.nz / 8) >= kStagedMinBlocks) {
      const int cz = staged_cz(cols, g.nz);
      const dim3 sgrid(cols * ((g.nz + cz - 1) / cz));
      if (t == LMR_BF16)
        hipLaunchKernelGGL((k_update_staged<uint16_t, MODE>), sgrid, dim3(kSNT), 0, s,
                           static_cast<const uint16_t*>(M), g, st, G, U0, U1, u_in, u_out,
                           r, lambda, eps, Mw, dMw, cz, ex);
      else
        hipLaunchKernelGGL((k_update_staged<float, MODE>), sgrid, dim3(kSNT), 0, s,
                           static_cast<const float*>(M), g, st, G, U0, U1, u_in, u_out, r,
                           lambda, eps, Mw, dMw, cz, ex);
      return hipGetLastError();
    }
  }
  const dim3 grid((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY, (g.nz + kUpdZ - 1) / kUpdZ);
  if (t == LMR_BF16)
    hipLaunchKernelGGL((k_update<uint16_t, MODE>), grid, blk, 0, s,
                       static_cast<const uint16_t*>(M), g, st, G, U0, U1, u_in, u_out,
                       r, lambda, eps, p.compositive, Mw, dMw, ex);
  else
    hipLaunchKernelGGL((k_update<float, MODE>), grid, blk, 0, s,
                       static_cast<const float*>(M), g, st, G, U0, U1, u_in, u_out, r,
                       lambda, eps, p.compositive, Mw, dMw, ex);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_update(const void* M, lmr_dtype t, const Geom& g,
                         const lmr_params& p, const DevState* st, const float* G,
                         float* U0, float* U1, const float* u_in, float* u_out,
                         double r, double lambda, float* Mw, float* dMw, hipStream_t s,
                         const StepExtra* extra) {
  const StepExtra ex = extra ? *extra : StepExtra{};
  switch (ex.mode) {
    case 0:
      return update_mode<0>(M, t, g, p, st, G, U0, U1, u_in, u_out, r, lambda, Mw, dMw, s, ex);
    case 1:
      return update_mode<1>(M, t, g, p, st, G, U0, U1, u_in, u_out, r, lambda, Mw, dMw, s, ex);
    case 2:
      if (!st) return hipErrorInvalidValue;  // the moments' step count lives in the state
      return update_mode<2>(M, t, g, p, st, G, U0, U1, u_in, u_out, r, lambda, Mw, dMw, s, ex);
    case 3:
      return update_mode<3>(M, t, g, p, st, G, U0, U1, u_in, u_out, r, lambda, Mw, dMw, s, ex);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_tile_hessian(const float* G, const Geom& g, int k, double* H,
                               const DevState* st, int need, hipStream_t s) {
  const int tx = (g.nx + k - 1) / k, ty = (g.ny + k - 1) / k, tz = (g.nz + k - 1) / k;
  const int n = tx * ty * tz;
  hipLaunchKernelGGL(k_tile_hessian, dim3((n + 255) / 256), dim3(256), 0, s, G, g, k, tx, ty,
                     n, H, st, need);
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
