// Per-pair launches of the three stencils of an LM attempt (stencil.h):
// LNCC forward (P2), LNCC + warp backward (P4) and Gaussian smoothing (P5).
// One block per tile; block ids are remapped so that each XCD receives a
// contiguous range of tiles and shares their halos in its L2.
#include <algorithm>

#include "decide.h"
#include "pass_decision.h"
#include "stencil.h"

namespace lmr {

namespace {

constexpr int kTY = 8;

// Waves per SIMD a stencil instantiation must leave register room for
// (measured choices; the others keep the compiler's own):
// * forward pass, BF16 images, compensated FP32 sums: 130 VGPRs left alone,
//   two above the 128 that allow four waves; asked for four, the compiler
//   fits it in 128 without spilling (200 -> 151 us at 160x192x224);
// * backward pass, BF16 images, FP64 sums: 156 VGPRs left alone; at four
//   waves nine VGPRs spill to scratch, and the attempt is still 5 % faster.
template <class P>
struct StencilWaves {
  static constexpr int value = 1;
};
template <int NT>
struct StencilWaves<FwdPol<uint16_t, NT, F32C>> {
  static constexpr int value = 4;
};
template <>
struct StencilWaves<BwdPol<uint16_t, double>> {
  static constexpr int value = 4;
};

// The decision of the attempt inside a pass of NT threads (pass_decision.h):
// every block reduces the partials and decides on the pair state st; block 0
// stores the result in pd.next.  Returns the decided state, in LDS.
template <int NT>
__device__ const DevState* decide_in_pass(const DevState* st, const PassDecision& pd) {
  __shared__ double sh[NT];
  __shared__ DevState s_next;
  DevState cur;
  if (threadIdx.x == 0) cur = *st;
  const double S = reduce_partials<NT>(pd.partials, pd.nparts, sh);
  if (threadIdx.x == 0) {
    const DevState n = decide_next(cur, -S / static_cast<double>(pd.N), pd.dp, pd.force);
    if (blockIdx.x == 0) *pd.next = n;
    s_next = n;
  }
  __syncthreads();
  return &s_next;
}

// Whether a block of a pass runs, and the state it runs on (rs; null without
// a pair state).  need: 0 always run, 1 skip a frozen pair, 2 run only after
// an acceptance.  DEC: the pass takes the decision first and runs on the
// decided state.  pd.commit: block 0 first stores st there.
template <int NT, bool DEC>
__device__ __forceinline__ bool pass_state(const DevState* st, int need,
                                           const PassDecision& pd, const DevState*& rs) {
  if constexpr (DEC) {
    rs = decide_in_pass<NT>(st, pd);
    return rs->accepted != 0;
  } else {
    rs = st;
    if (pd.commit && blockIdx.x == 0 && threadIdx.x == 0) *pd.commit = *st;
    if (st && need) {
      if (st->stalled) return false;
      if (need == 2 && !st->accepted) return false;
    }
    return true;
  }
}

// A marching pass that takes the decision is held to the waves per SIMD the
// pass has without it (left alone, the compiler gives the decision's registers
// to the stencil and loses a wave): four with FP64 sums, three with
// compensated FP32 sums (which spill at four).
template <class P>
struct DecidingWaves {
  static constexpr int value = std::is_same<typename P::Acc, F32C>::value ? 3 : 4;
};

template <int R, int TY, class P, bool DEC>
__global__ void __launch_bounds__(kTX* TY)
    __attribute__((amdgpu_waves_per_eu(DEC ? DecidingWaves<P>::value
                                           : StencilWaves<P>::value)))
    k_stencil(const P pol, Geom g, Tiling t, const DevState* st, int need, PassDecision pd) {
  const DevState* rs;
  if (!pass_state<kTX * TY, DEC>(st, need, pd, rs)) return;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  int x0, y0, z0;
  tile_origin(t, tile, TY, x0, y0, z0);
  typename P::Local loc = pol.begin_block(rs);
  stencil_tile<R, TY>(pol, g, x0, y0, z0, min(z0 + t.cz, g.nz), loc);
  pol.end_tile(loc, tile);  // partials in tile order, as in the batched form
}

// The same stencil on TZ x kT3 x kT3 bricks (small volumes; stencil.h).
template <int R, class P, int TZ, bool DEC>
__global__ void __launch_bounds__(kCubeThreads)
    __attribute__((amdgpu_waves_per_eu(DEC ? 4 : 1)))
    k_cube(const P pol, Geom g, int cubes_x, int cubes_y, const DevState* st, int need,
           PassDecision pd) {
  const DevState* rs;
  if (!pass_state<kCubeThreads, DEC>(st, need, pd, rs)) return;
  __shared__ CubeLds<R, P, TZ> sm;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int x0 = (b % cubes_x) * kT3, y0 = ((b / cubes_x) % cubes_y) * kT3;
  const int z0 = (b / (cubes_x * cubes_y)) * TZ;
  typename P::Local loc = pol.begin_block(rs);
  stencil_cube<R, TZ>(pol, g, x0, y0, z0, loc, sm);
  pol.end_tile(loc, b);
}

}  // namespace

// Chunk length of the march.  A launch runs its blocks in rounds of
// 4 x CUs co-resident ones (the forward and backward passes' occupancy with
// FP64 sums and window 7; the smoothing pass holds 8 per CU but is bound by
// memory and runs fastest on the same chunks), and each block of a round
// marches its chunk plus the 2R halo planes, so a launch lasts about
// ceil(tiles / (4 CUs)) x (cz + 2R) plane steps.  Among the chunk lengths
// not below make_tiling's floor, take the one that minimises this (the longer
// chunk on a tie).  It does not depend on the kernel: a box sum's rounding
// depends on where its chunk starts, and the batched form reproduces a pair's
// run by using the same tiling for all passes.
Tiling march_tiling(const Geom& g, int R) {
  Tiling t = make_tiling(g.nz, g.ny, g.nx, kTY);
  const long long cols = (long long)t.tiles_x * t.tiles_y;
  const long long cap = 4LL * device_cus();
  const int floor_cz = std::min(march_floor_cz(cols, g.nz), g.nz);
  long long best = -1;
  for (int n = 1; n <= g.nz; ++n) {
    const int cz = (g.nz + n - 1) / n;
    if (cz < floor_cz) break;
    const int chunks = (g.nz + cz - 1) / cz;
    if (chunks != n) continue;  // the same chunk length as a smaller n
    const long long cost = ((cols * chunks + cap - 1) / cap) * (cz + 2 * R);
    if (best < 0 || cost < best) {
      best = cost;
      t.cz = cz;
      t.nchunks = chunks;
    }
  }
  return t;
}

namespace {

// The forward policy's block reduction is sized for its block: one policy
// type serves both forms, so both forms launch blocks of the same size.
static_assert(kTX * kTY == kCubeThreads, "marching tiles and cubes share FwdPol<T, 256>");

// Volumes of at most this many voxels run on cubes under LMR_STENCIL_AUTO
// (the half- and quarter-resolution levels of a brain-sized pair).
constexpr long long kCubeMaxVoxels = 1LL << 20;

bool use_cubes(const Geom& g, const lmr_params& p) {
  return p.stencil == LMR_STENCIL_CUBE ||
         (p.stencil == LMR_STENCIL_AUTO && g.N <= kCubeMaxVoxels);
}

// Bricks are 8 planes deep, or 4 where 8-plane bricks would give fewer than
// kCubeSplitBelow blocks (the quarter-resolution level): there each block's
// own latency is the launch's, and halving its work halves that.
constexpr int kCubeSplitBelow = 512;

int cube_columns(const Geom& g) { return ((g.nx + kT3 - 1) / kT3) * ((g.ny + kT3 - 1) / kT3); }

int cube_tz(const Geom& g) {
  return cube_columns(g) * ((g.nz + 7) / 8) < kCubeSplitBelow ? 4 : 8;
}

int cube_count(const Geom& g) {
  const int tz = cube_tz(g);
  return cube_columns(g) * ((g.nz + tz - 1) / tz);
}

template <class P, int R, bool DEC = false>
hipError_t run(const P& pol, const Geom& g, bool cubes, const DevState* st, int need,
               hipStream_t s, const PassDecision& pd = PassDecision{}) {
  if constexpr (DEC && R > kPassDecisionMaxRadius) {
    return hipErrorInvalidValue;  // wider windows keep the decision kernel
  } else {
    if (cubes) {
      const int cx = (g.nx + kT3 - 1) / kT3, cy = (g.ny + kT3 - 1) / kT3;
      if (cube_tz(g) == 4)
        hipLaunchKernelGGL((k_cube<R, P, 4, DEC>), dim3(cube_count(g)), dim3(kCubeThreads),
                           0, s, pol, g, cx, cy, st, need, pd);
      else if constexpr (DEC)
        return hipErrorInvalidValue;  // 8-plane bricks keep the decision kernel
      else
        hipLaunchKernelGGL((k_cube<R, P, 8, false>), dim3(cube_count(g)),
                           dim3(kCubeThreads), 0, s, pol, g, cx, cy, st, need, pd);
      return hipGetLastError();
    }
    const Tiling t = march_tiling(g, R);
    hipLaunchKernelGGL((k_stencil<R, kTY, P, DEC>), dim3(t.tiles()), dim3(kTX * kTY), 0, s,
                       pol, g, t, st, need, pd);
    return hipGetLastError();
  }
}

template <class P, bool DEC = false>
hipError_t run_box(const P& pol, int window, const Geom& g, bool cubes, const DevState* st,
                   int need, hipStream_t s, const PassDecision& pd = PassDecision{}) {
  switch (window / 2) {
    case 1: return run<P, 1, DEC>(pol, g, cubes, st, need, s, pd);
    case 2: return run<P, 2, DEC>(pol, g, cubes, st, need, s, pd);
    case 3: return run<P, 3, DEC>(pol, g, cubes, st, need, s, pd);
    case 4: return run<P, 4, DEC>(pol, g, cubes, st, need, s, pd);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, typename Acc>
hipError_t fstat_t(const T* F, const Geom& g, const lmr_params& p, double* fstat,
                   hipStream_t s) {
  FStatPol<T, Acc> pol;
  pol.F = F;
  pol.fstat = fstat;
  pol.N = static_cast<int>(g.N);
  pol.inv_n = 1.0 / ((double)p.window * p.window * p.window);
  return run_box(pol, p.window, g, use_cubes(g, p), nullptr, 0, s);
}

template <typename T, typename Acc>
hipError_t fwd_t(const T* F, const float* Mw, const double* fstat, const Geom& g,
                 const lmr_params& p, const DevState* st, float* maps, double* partials,
                 int nparts, float* cc, hipStream_t s) {
  if (fwd_num_blocks(g, p) != nparts) return hipErrorInvalidValue;
  FwdPol<T, kTX * kTY, Acc> pol;
  pol.F = F;
  pol.Mw = Mw;
  pol.fstat = fstat;
  pol.maps = maps;
  pol.cc = cc;
  pol.partials = partials;
  pol.N = static_cast<int>(g.N);
  pol.inv_n = 1.0 / ((double)p.window * p.window * p.window);
  pol.eps = p.cc_eps;
  return run_box(pol, p.window, g, use_cubes(g, p), st, 1, s);
}

template <typename T, typename Acc>
hipError_t bwd_t(const T* F, const T* M, const float* Mw, const float* maps,
                 const Geom& g, const lmr_params& p, const DevState* st,
                 const float* U0, const float* U1, const float* ue, const float* dMw,
                 float* graw, hipStream_t s, const PassDecision* pd = nullptr) {
  BwdPol<T, Acc> pol;
  pol.F = F;
  pol.M = M;
  pol.Mw = Mw;
  pol.maps = maps;
  pol.U0 = U0;
  pol.U1 = U1;
  pol.u_explicit = ue;
  pol.dMw = dMw;
  pol.graw = graw;
  pol.g = g;
  pol.inv_n = 1.0 / ((double)p.window * p.window * p.window);
  if (pd) return run_box<BwdPol<T, Acc>, true>(pol, p.window, g, use_cubes(g, p), st, 2, s, *pd);
  return run_box(pol, p.window, g, use_cubes(g, p), st, 2, s);
}

template <int R>
hipError_t smooth_r(const float* in, float* out, const Geom& g, const lmr_params& p,
                    const DevState* st, hipStream_t s, DevState* commit = nullptr) {
  SmoothPol<R> pol;
  pol.in = in;
  pol.out = out;
  pol.N = static_cast<int>(g.N);
  gauss_taps<R>(p.grad_sigma, pol.w);
  PassDecision pd{};
  pd.commit = commit;
  return run<SmoothPol<R>, R>(pol, g, use_cubes(g, p), st, 2, s, pd);
}

}  // namespace

int brick_depth(const Geom& g, const lmr_params& p) {
  return use_cubes(g, p) ? cube_tz(g) : 0;
}

int brick_count(const Geom& g, int tz) { return cube_columns(g) * ((g.nz + tz - 1) / tz); }

int fwd_num_blocks(const Geom& g, const lmr_params& p) {
  return use_cubes(g, p) ? cube_count(g) : march_tiling(g, p.window / 2).tiles();
}

int gauss_radius(double sigma) {
  if (!(sigma > 0.0)) return 0;
  return (int)ceil(3.0 * sigma - 1e-12);
}

// The box sums accumulate in FP64 (LMR_ACC_F64) or in compensated FP32
// (LMR_ACC_F32C); the image type picks the loads.
hipError_t launch_fstat(const void* F, lmr_dtype t, const Geom& g, const lmr_params& p,
                        double* fstat, hipStream_t s) {
  if (t == LMR_BF16) {
    const uint16_t* f = static_cast<const uint16_t*>(F);
    return p.accum == LMR_ACC_F32C ? fstat_t<uint16_t, F32C>(f, g, p, fstat, s)
                                   : fstat_t<uint16_t, double>(f, g, p, fstat, s);
  }
  const float* f = static_cast<const float*>(F);
  return p.accum == LMR_ACC_F32C ? fstat_t<float, F32C>(f, g, p, fstat, s)
                                 : fstat_t<float, double>(f, g, p, fstat, s);
}

hipError_t launch_fwd(const void* F, lmr_dtype t, const float* Mw, const double* fstat,
                      const Geom& g, const lmr_params& p, const DevState* st, float* maps,
                      double* partials, int nparts, float* cc_map, hipStream_t s) {
  if (t == LMR_BF16) {
    const uint16_t* f = static_cast<const uint16_t*>(F);
    return p.accum == LMR_ACC_F32C
               ? fwd_t<uint16_t, F32C>(f, Mw, fstat, g, p, st, maps, partials, nparts, cc_map,
                                       s)
               : fwd_t<uint16_t, double>(f, Mw, fstat, g, p, st, maps, partials, nparts,
                                         cc_map, s);
  }
  const float* f = static_cast<const float*>(F);
  return p.accum == LMR_ACC_F32C
             ? fwd_t<float, F32C>(f, Mw, fstat, g, p, st, maps, partials, nparts, cc_map, s)
             : fwd_t<float, double>(f, Mw, fstat, g, p, st, maps, partials, nparts, cc_map,
                                    s);
}

hipError_t launch_bwd(const void* F, const void* M, lmr_dtype t, const float* Mw,
                      const float* maps, const Geom& g, const lmr_params& p,
                      const DevState* st, const float* U0, const float* U1,
                      const float* ue, const float* dMw, float* graw, hipStream_t s) {
  if (t == LMR_BF16) {
    const uint16_t *f = static_cast<const uint16_t*>(F), *m = static_cast<const uint16_t*>(M);
    return p.accum == LMR_ACC_F32C
               ? bwd_t<uint16_t, F32C>(f, m, Mw, maps, g, p, st, U0, U1, ue, dMw, graw, s)
               : bwd_t<uint16_t, double>(f, m, Mw, maps, g, p, st, U0, U1, ue, dMw, graw, s);
  }
  const float *f = static_cast<const float*>(F), *m = static_cast<const float*>(M);
  return p.accum == LMR_ACC_F32C
             ? bwd_t<float, F32C>(f, m, Mw, maps, g, p, st, U0, U1, ue, dMw, graw, s)
             : bwd_t<float, double>(f, m, Mw, maps, g, p, st, U0, U1, ue, dMw, graw, s);
}

hipError_t launch_smooth(const float* graw, const Geom& g, const lmr_params& p,
                         const DevState* st, float* out, hipStream_t s) {
  switch (gauss_radius(p.grad_sigma)) {
    case 0: return smooth_r<0>(graw, out, g, p, st, s);
    case 1: return smooth_r<1>(graw, out, g, p, st, s);
    case 2: return smooth_r<2>(graw, out, g, p, st, s);
    case 3: return smooth_r<3>(graw, out, g, p, st, s);
    case 4: return smooth_r<4>(graw, out, g, p, st, s);
    case 5: return smooth_r<5>(graw, out, g, p, st, s);
    case 6: return smooth_r<6>(graw, out, g, p, st, s);
    default: return hipErrorInvalidValue;
  }
}

bool bwd_takes_decision(const Geom& g, const lmr_params& p, int nparts) {
  return nparts <= kPassDecisionMaxParts && p.window / 2 <= kPassDecisionMaxRadius &&
         !(use_cubes(g, p) && cube_tz(g) == 8);
}

hipError_t launch_bwd_decide(const void* F, const void* M, lmr_dtype t, const float* Mw,
                             const float* maps, const Geom& g, const lmr_params& p,
                             const DevState* st, const float* U0, const float* U1,
                             const float* dMw, float* graw, const PassDecision& pd,
                             hipStream_t s) {
  if (!st || !pd.partials || !pd.next || !bwd_takes_decision(g, p, pd.nparts))
    return hipErrorInvalidValue;
  if (t == LMR_BF16) {
    const uint16_t *f = static_cast<const uint16_t*>(F), *m = static_cast<const uint16_t*>(M);
    return p.accum == LMR_ACC_F32C
               ? bwd_t<uint16_t, F32C>(f, m, Mw, maps, g, p, st, U0, U1, nullptr, dMw, graw,
                                       s, &pd)
               : bwd_t<uint16_t, double>(f, m, Mw, maps, g, p, st, U0, U1, nullptr, dMw, graw,
                                         s, &pd);
  }
  const float *f = static_cast<const float*>(F), *m = static_cast<const float*>(M);
  return p.accum == LMR_ACC_F32C
             ? bwd_t<float, F32C>(f, m, Mw, maps, g, p, st, U0, U1, nullptr, dMw, graw, s, &pd)
             : bwd_t<float, double>(f, m, Mw, maps, g, p, st, U0, U1, nullptr, dMw, graw, s,
                                    &pd);
}

hipError_t launch_smooth_commit(const float* graw, const Geom& g, const lmr_params& p,
                                const DevState* next, DevState* st, float* out,
                                hipStream_t s) {
  if (!next || !st) return hipErrorInvalidValue;
  switch (gauss_radius(p.grad_sigma)) {
    case 0: return smooth_r<0>(graw, out, g, p, next, s, st);
    case 1: return smooth_r<1>(graw, out, g, p, next, s, st);
    case 2: return smooth_r<2>(graw, out, g, p, next, s, st);
    case 3: return smooth_r<3>(graw, out, g, p, next, s, st);
    case 4: return smooth_r<4>(graw, out, g, p, next, s, st);
    case 5: return smooth_r<5>(graw, out, g, p, next, s, st);
    case 6: return smooth_r<6>(graw, out, g, p, next, s, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lmr
