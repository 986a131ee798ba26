// Batched form: every pair of a batch of uneven-size pairs advances by one
// LM attempt in ONE persistent launch.  The grid holds only as many blocks as
// fit on the GPU at once (occupancy query); the blocks sweep the work list of
// each phase and meet at a grid barrier between phases:
//
//   P1 update     work items: staged-update tiles (32x8 columns over a z-chunk)
//   P2 lncc_fwd   work items: stencil tiles of a pair (partial of cc per tile):
//                 marching tiles, or 4-plane bricks for the pairs a stand-alone
//                 context runs on them
//   P3 decide     work items: pairs (one block reduces a pair's partials)
//   P4 lncc_bwd   stencil tiles of the pairs whose candidate was accepted
//   P5 smooth     stencil tiles of the pairs whose candidate was accepted
//
// Each pair keeps its own device state (lambda, loss history, decision), so
// pairs accept, reject and freeze independently.  A barrier wait is bounded
// in time: past the limit the kernel records an error and every block leaves
// (later launches return at once), so a residency mistake cannot hang the
// device.
#pragma once

#include <type_traits>

#include "decide.h"
#include "lmr_batch.h"
#include "stencil.h"
#include "update.h"

namespace lmr {

// Included by one translation unit per box-sum accumulator (k_batch.hip:
// FP64, k_batch_f32c.hip: compensated FP32), so that the two sets of
// instantiations compile in parallel.
namespace {

constexpr int kTY = 8;
constexpr int kNT = kTX * kTY;
static_assert(kBatchUpdateTX == kSX && kBatchUpdateTY == kSY && kNT == kSNT,
              "update work items are staged-update tiles of one block");

// Grid-wide barrier among `nblocks` co-resident blocks (two-level arrival on
// monotonic counters, see BatchCtl).  A wait longer than `timeout` ticks of
// the device's constant-rate wall clock records error 1.  With ticket > 0
// (at the first barrier of a launch: 1 + the block's ticket from count_in),
// a wait longer than start_timeout ticks while some block of this launch has
// not even started records error 2: that block is not on the GPU (other work
// holds its resources), so waiting longer would only wait for that work.
// The started counts are kept per group like the arrivals, so that the
// blocks' start does not queue on one cache line.  Returns false when this
// wait failed or another block reported a failure.
__device__ __noinline__ bool all_started(BatchCtl* ctl, unsigned nblocks,
                                         unsigned long long ticket) {
  // this block's launch (1, 2, ... since the reset) from its ticket
  const unsigned grp = blockIdx.x % kBarGroups;
  const unsigned long long launch =
      ticket / ((nblocks + kBarGroups - 1 - grp) / kBarGroups) + 1;
  for (int g = 0; g < kBarGroups; ++g) {
    const unsigned long long in_g = (nblocks + kBarGroups - 1 - g) / kBarGroups;
    if (in_g && __hip_atomic_load(&ctl->started[g].v, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT) < launch * in_g)
      return false;
  }
  return true;
}
__device__ bool grid_sync(BatchCtl* ctl, unsigned nblocks, unsigned long long timeout,
                          unsigned long long ticket = 0,
                          unsigned long long start_timeout = 0) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    // release: this block's results are written back to where blocks on the
    // other chiplets read them, before its arrival is counted
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned grp = blockIdx.x % kBarGroups;
    const unsigned long long in_grp = (nblocks + kBarGroups - 1 - grp) / kBarGroups;
    const unsigned long long ngrp = nblocks < (unsigned)kBarGroups ? nblocks : kBarGroups;
    const unsigned long long a = atomicAdd(&ctl->group[grp].v, 1ull);
    const unsigned long long epoch = a / in_grp;  // barriers completed before this one
    bool release = false;
    if ((a + 1) % in_grp == 0) {
      const unsigned long long t = atomicAdd(&ctl->top.v, 1ull);
      if ((t + 1) % ngrp == 0) {
        __hip_atomic_fetch_add(&ctl->gen.v, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        release = true;
      }
    }
    int good = 1;
    if (!release) {
      const unsigned long long t0 = wall_clock64();
      // relaxed polls (an acquire per poll would invalidate this chiplet's L2
      // under the working blocks every time); the fence below acquires once
      while (__hip_atomic_load(&ctl->gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <=
             epoch) {
        const unsigned long long dt = wall_clock64() - t0;
        unsigned long long code = 0;
        if (dt > timeout)
          code = 1;
        else if (ticket && dt > start_timeout && !all_started(ctl, nblocks, ticket - 1))
          code = 2;
        if (code) {
          good = 0;
          atomicCAS(&ctl->error.v, 0ull, code);  // the first failure is reported
          break;
        }
        if (__hip_atomic_load(&ctl->error.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(4);
      }
    }
    // acquire: stale lines of this chiplet's caches are dropped, so the
    // results of the other blocks are read from memory
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = good && __hip_atomic_load(&ctl->error.v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) == 0;
  }
  __syncthreads();
  return ok != 0;
}

// Counts the calling block in on its group's started line and returns its
// ticket (kept out of line: inlined at the kernel's start it raised the
// register count of every instantiation by 35-70 VGPRs).  Test hook: with
// late != 0, block 0 first waits twice the co-residency limit, as a block
// that was not on the GPU would (bounded wait).
__device__ __noinline__ unsigned long long count_in(BatchCtl* ctl, int late,
                                                    unsigned long long start_timeout) {
  if (late && blockIdx.x == 0) {
    const unsigned long long t0 = wall_clock64();
    while (wall_clock64() - t0 < 2 * start_timeout) __builtin_amdgcn_s_sleep(8);
  }
  return atomicAdd(&ctl->started[blockIdx.x % kBarGroups].v, 1ull);
}

// A state field written earlier in this launch by another block: read with a
// device-scope atomic so that no cached copy is used.
__device__ __forceinline__ int fresh(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// origin of brick `b` of a pair (x fastest, then y, then z), as a stand-alone
// context numbers its bricks
__device__ __forceinline__ void brick_origin(const Geom& g, int b, int& x0, int& y0,
                                             int& z0) {
  const int cx = (g.nx + kT3 - 1) / kT3, cy = (g.ny + kT3 - 1) / kT3;
  x0 = (b % cx) * kT3;
  y0 = ((b / cx) % cy) * kT3;
  z0 = (b / (cx * cy)) * kBatchBrickTZ;
}

// pair owning work item `it` of a list whose per-pair offsets are first[p]
__device__ __forceinline__ int owner(const BatchPair* __restrict__ pairs, int npairs,
                                     int it, bool tiles) {
  int p = 0;
  for (int k = 1; k < npairs; ++k)
    if ((tiles ? pairs[k].tile0 : pairs[k].utile0) <= it) p = k;
  return p;
}

// LDS of a brick phase, in the kernels that run bricks (BR = 1) only: the
// brick path needs more registers, so pairs that all march keep a kernel
// without it.
template <int R, class P, int BR>
using BrickLds = std::conditional_t<BR != 0, CubeLds<R, P, kBatchBrickTZ>, char>;

// One work item of each phase, shared by the persistent kernel (a grid-stride
// loop per phase, grid barriers between them) and the per-phase kernels (one
// item per block, k_batch_phases.hip).  FORM: 0 marching pairs only, 1
// brick pairs only, 2 either; an item of a pair of the other form is skipped.

// P1: closed form, compositive integration, candidate warp (and its
// derivative, which P4 reads), one staged tile per work item
template <typename T>
__device__ __forceinline__ void update_item(const BatchPair* __restrict__ pairs, int npairs,
                                            int it, StagedLds& lds) {
  const BatchPair& P = pairs[owner(pairs, npairs, it, false)];
  if (P.st->stalled) return;
  UpdateArgs a = update_args_from_state(P.st, P.U0, P.U1, P.G, P.Mw, P.eps, P.compositive);
  a.dMw = P.graw;
  const int local = it - P.utile0;
  const int tx = (P.g.nx + kSX - 1) / kSX, ty = (P.g.ny + kSY - 1) / kSY;
  const int bx = (local % tx) * kSX, by = ((local / tx) % ty) * kSY;
  const int z0 = (local / (tx * ty)) * P.ucz;
  const int z1 = min(z0 + P.ucz, P.g.nz);
  if (P.compositive) {
    staged_update_tile(static_cast<const T*>(P.M), P.g, a, point_step(a, P.g), bx, by, z0, z1,
                       lds);
  } else {
    const int x = bx + static_cast<int>(threadIdx.x) % kSX;
    const int y = by + static_cast<int>(threadIdx.x) / kSX;
    if (x < P.g.nx && y < P.g.ny)
      for (int z = z0; z < z1; ++z) update_voxel(static_cast<const T*>(P.M), P.g, a, x, y, z);
  }
}

// the stencil of one work item of pair P with policy pol: a brick or a
// marching tile (LM, LB: the LDS of either form; char where not compiled)
template <int R, int FORM, class Pol, class LM, class LB>
__device__ __forceinline__ void stencil_item(const Pol& pol, const BatchPair& P, int local,
                                             typename Pol::Local& loc, LM& lm, LB& lb) {
  int x0, y0, z0;
  if (FORM != 0 && P.bricks) {
    if constexpr (FORM != 0) {
      brick_origin(P.g, local, x0, y0, z0);
      __syncthreads();  // the previous brick's last LDS reads are done
      stencil_cube<R, kBatchBrickTZ>(pol, P.g, x0, y0, z0, loc, lb);
    }
  } else {
    if constexpr (FORM != 1) {
      tile_origin(P.t, local, kTY, x0, y0, z0);
      stencil_tile<R, kTY>(pol, P.g, x0, y0, z0, min(z0 + P.t.cz, P.g.nz), loc, lm);
    }
  }
}

template <int FORM>
__device__ __forceinline__ bool other_form(const BatchPair& P) {
  return (FORM == 0 && P.bricks) || (FORM == 1 && !P.bricks);
}

// P2: LNCC forward, one partial of cc per tile
template <int RB, typename T, typename Acc, int FORM, class LM, class LB>
__device__ __forceinline__ void fwd_item(const BatchPair* __restrict__ pairs, int npairs,
                                         int it, LM& lm, LB& lb) {
  const BatchPair& P = pairs[owner(pairs, npairs, it, true)];
  if (P.st->stalled || other_form<FORM>(P)) return;
  FwdPol<T, kNT, Acc> pol;
  pol.F = static_cast<const T*>(P.F);
  pol.Mw = P.Mw;
  pol.fstat = P.fstat;
  pol.maps = P.maps;
  pol.cc = nullptr;
  pol.partials = P.partials;
  pol.N = static_cast<int>(P.g.N);
  pol.inv_n = P.inv_n;
  pol.eps = P.cc_eps;
  const int local = it - P.tile0;
  auto loc = pol.begin_block(P.st);
  stencil_item<RB, FORM>(pol, P, local, loc, lm, lb);
  pol.end_tile(loc, local);
}

// P4: LNCC and warp backward of the accepted candidates
template <int RB, typename T, typename Acc, int FORM, class LM, class LB>
__device__ __forceinline__ void bwd_item(const BatchPair* __restrict__ pairs, int npairs,
                                         int it, LM& lm, LB& lb) {
  const BatchPair& P = pairs[owner(pairs, npairs, it, true)];
  if (fresh(&P.st->stalled) || !fresh(&P.st->accepted) || other_form<FORM>(P)) return;
  BwdPol<T, Acc> pol;
  pol.F = static_cast<const T*>(P.F);
  pol.M = static_cast<const T*>(P.M);
  pol.Mw = P.Mw;
  pol.maps = P.maps;
  pol.U0 = P.U0;
  pol.U1 = P.U1;
  pol.u_explicit = fresh(&P.st->cur) ? P.U1 : P.U0;  // the accepted candidate
  pol.dMw = P.graw;  // stored there by P1 for the candidate
  pol.graw = P.graw;
  pol.g = P.g;
  pol.inv_n = P.inv_n;
  auto loc = pol.begin_block(nullptr);
  stencil_item<RB, FORM>(pol, P, it - P.tile0, loc, lm, lb);
}

// P5: Gaussian smoothing of the new gradient
template <int RG, int FORM, class LM, class LB>
__device__ __forceinline__ void smooth_item(const BatchPair* __restrict__ pairs, int npairs,
                                            int it, LM& lm, LB& lb) {
  const BatchPair& P = pairs[owner(pairs, npairs, it, true)];
  if (fresh(&P.st->stalled) || !fresh(&P.st->accepted) || other_form<FORM>(P)) return;
  SmoothPol<RG> pol;
  pol.in = P.graw;
  pol.out = P.G;
  pol.N = static_cast<int>(P.g.N);
#pragma unroll
  for (int k = 0; k <= 2 * RG; ++k) pol.w[k] = P.gw[k];
  auto loc = pol.begin_block(P.st);
  stencil_item<RG, FORM>(pol, P, it - P.tile0, loc, lm, lb);
}

template <int RB, int RG, typename T, typename Acc, int BR>
__global__ void __launch_bounds__(kNT)
    k_batch_attempt(const BatchPair* __restrict__ pairs, int npairs, int n_update_items,
                    int n_tiles, BatchCtl* ctl, DecideParams dp,
                    unsigned long long timeout, unsigned long long start_timeout,
                    int missing) {
  constexpr int FORM = BR ? 2 : 0;
  const int nb = gridDim.x;
  // the phases are separated by grid barriers, so their LDS is overlaid
  __shared__ union {
    StagedLds upd;
    StencilLds<RB, kTY, FwdPol<T, kNT, Acc>> fwd;
    StencilLds<RB, kTY, BwdPol<T, Acc>> bwd;
    StencilLds<RG, kTY, SmoothPol<RG>> smo;
    BrickLds<RB, FwdPol<T, kNT, Acc>, BR> fwd_b;
    BrickLds<RB, BwdPol<T, Acc>, BR> bwd_b;
    BrickLds<RG, SmoothPol<RG>, BR> smo_b;
  } lds;
  // after a barrier failure every later launch returns at once
  if (__hip_atomic_load(&ctl->error.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  // count this block in; launches of one stream do not overlap, so the
  // ticket tells which launch this is (thread 0 alone uses it)
  unsigned long long ticket = 0;
  if (threadIdx.x == 0) ticket = count_in(ctl, missing, start_timeout) + 1;

  for (int it = blockIdx.x; it < n_update_items; it += nb)
    update_item<T>(pairs, npairs, it, lds.upd);
  // P1 wrote only candidates (the accepted fields, the smoothed gradients
  // and the states are untouched), so a launch that fails here leaves every
  // pair as the previous launch left it
  if (!grid_sync(ctl, nb, timeout, ticket, start_timeout)) return;
  for (int it = blockIdx.x; it < n_tiles; it += nb)
    fwd_item<RB, T, Acc, FORM>(pairs, npairs, it, lds.fwd, lds.fwd_b);
  if (!grid_sync(ctl, nb, timeout)) return;
  // P3: per-pair FP64 reduction and decision
  for (int p = blockIdx.x; p < npairs; p += nb) {
    const BatchPair& P = pairs[p];
    decide_block<kNT>(P.st, P.partials, P.ntiles, P.g.N, dp, 0, -1, 0.0, nullptr);
  }
  if (!grid_sync(ctl, nb, timeout)) return;
  for (int it = blockIdx.x; it < n_tiles; it += nb)
    bwd_item<RB, T, Acc, FORM>(pairs, npairs, it, lds.bwd, lds.bwd_b);
  if (!grid_sync(ctl, nb, timeout)) return;
  for (int it = blockIdx.x; it < n_tiles; it += nb)
    smooth_item<RG, FORM>(pairs, npairs, it, lds.smo, lds.smo_b);
}

template <int RB, int RG, typename T, typename Acc, int BR>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&k_batch_attempt<RB, RG, T, Acc, BR>);
}

template <typename T, typename Acc, int BR>
const void* kernel_for(int rb, int rg) {
#define LMR_RG(RBV)                                    \
  switch (rg) {                                        \
    case 0: return kernel_ptr<RBV, 0, T, Acc, BR>();   \
    case 1: return kernel_ptr<RBV, 1, T, Acc, BR>();   \
    case 2: return kernel_ptr<RBV, 2, T, Acc, BR>();   \
    case 3: return kernel_ptr<RBV, 3, T, Acc, BR>();   \
    case 4: return kernel_ptr<RBV, 4, T, Acc, BR>();   \
    default: return nullptr;                           \
  }
  switch (rb) {
    case 1: LMR_RG(1)
    case 2: LMR_RG(2)
    case 3: LMR_RG(3)
    case 4: LMR_RG(4)
    default: return nullptr;
  }
#undef LMR_RG
}

template <typename Acc, int BR>
const void* batch_kernel_for(lmr_dtype t, int box_radius, int gauss_radius) {
  return t == LMR_BF16 ? kernel_for<uint16_t, Acc, BR>(box_radius, gauss_radius)
                       : kernel_for<float, Acc, BR>(box_radius, gauss_radius);
}

}  // namespace

}  // namespace lmr
