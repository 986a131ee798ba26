// Batched form without the persistent kernel: each phase of an attempt is one
// launch over the work items of all pairs (one item per block), so the
// kernel boundaries order the phases instead of grid barriers, and every
// phase kernel has the registers, and so the occupancy, of its own work
// (batch_attempt.h holds the items).  A phase whose pairs run on both forms
// is launched once per form, each launch skipping the other form's items.
#include "batch_attempt.h"

namespace lmr {

namespace {

template <typename T>
__global__ void __launch_bounds__(kNT) k_bp_update(const BatchPair* __restrict__ pairs,
                                                   int npairs) {
  __shared__ StagedLds lds;
  update_item<T>(pairs, npairs, blockIdx.x, lds);
}

__global__ void __launch_bounds__(kNT) k_bp_decide(const BatchPair* __restrict__ pairs,
                                                   DecideParams dp) {
  const BatchPair& P = pairs[blockIdx.x];
  decide_block<kNT>(P.st, P.partials, P.ntiles, P.g.N, dp, 0, -1, 0.0, nullptr);
}

// The LDS of a stencil phase kernel of one form.
template <int R, class Pol, int FORM>
using FormLds = std::conditional_t<FORM == 1, CubeLds<R, Pol, kBatchBrickTZ>,
                                   StencilLds<R, kTY, Pol>>;

template <int RB, typename T, typename Acc, int FORM>
__global__ void __launch_bounds__(kNT) k_bp_fwd(const BatchPair* __restrict__ pairs,
                                                int npairs) {
  __shared__ FormLds<RB, FwdPol<T, kNT, Acc>, FORM> lds;
  char none;
  if constexpr (FORM == 1)
    fwd_item<RB, T, Acc, 1>(pairs, npairs, blockIdx.x, none, lds);
  else
    fwd_item<RB, T, Acc, 0>(pairs, npairs, blockIdx.x, lds, none);
}

template <int RB, typename T, typename Acc, int FORM>
__global__ void __launch_bounds__(kNT) k_bp_bwd(const BatchPair* __restrict__ pairs,
                                                int npairs) {
  __shared__ FormLds<RB, BwdPol<T, Acc>, FORM> lds;
  char none;
  if constexpr (FORM == 1)
    bwd_item<RB, T, Acc, 1>(pairs, npairs, blockIdx.x, none, lds);
  else
    bwd_item<RB, T, Acc, 0>(pairs, npairs, blockIdx.x, lds, none);
}

template <int RG, int FORM>
__global__ void __launch_bounds__(kNT) k_bp_smooth(const BatchPair* __restrict__ pairs,
                                                   int npairs) {
  __shared__ FormLds<RG, SmoothPol<RG>, FORM> lds;
  char none;
  if constexpr (FORM == 1)
    smooth_item<RG, 1>(pairs, npairs, blockIdx.x, none, lds);
  else
    smooth_item<RG, 0>(pairs, npairs, blockIdx.x, lds, none);
}

struct PhaseLaunch {
  const BatchPair* pairs;
  int npairs, n_update_items, n_tiles;
  bool march, bricks;
  hipStream_t s;
};

template <int RB, typename T, typename Acc>
void launch_box(const PhaseLaunch& L, bool fwd) {
  const dim3 grid(L.n_tiles), blk(kNT);
  if (L.march) {
    if (fwd)
      hipLaunchKernelGGL((k_bp_fwd<RB, T, Acc, 0>), grid, blk, 0, L.s, L.pairs, L.npairs);
    else
      hipLaunchKernelGGL((k_bp_bwd<RB, T, Acc, 0>), grid, blk, 0, L.s, L.pairs, L.npairs);
  }
  if (L.bricks) {
    if (fwd)
      hipLaunchKernelGGL((k_bp_fwd<RB, T, Acc, 1>), grid, blk, 0, L.s, L.pairs, L.npairs);
    else
      hipLaunchKernelGGL((k_bp_bwd<RB, T, Acc, 1>), grid, blk, 0, L.s, L.pairs, L.npairs);
  }
}

template <int RG>
void launch_smooth_forms(const PhaseLaunch& L) {
  const dim3 grid(L.n_tiles), blk(kNT);
  if (L.march) hipLaunchKernelGGL((k_bp_smooth<RG, 0>), grid, blk, 0, L.s, L.pairs, L.npairs);
  if (L.bricks) hipLaunchKernelGGL((k_bp_smooth<RG, 1>), grid, blk, 0, L.s, L.pairs, L.npairs);
}

template <typename T, typename Acc>
hipError_t phases_t(const PhaseLaunch& L, int rb, int rg, const DecideParams& dp) {
  auto box = [&](bool fwd) -> bool {
    switch (rb) {
      case 1: launch_box<1, T, Acc>(L, fwd); return true;
      case 2: launch_box<2, T, Acc>(L, fwd); return true;
      case 3: launch_box<3, T, Acc>(L, fwd); return true;
      case 4: launch_box<4, T, Acc>(L, fwd); return true;
      default: return false;
    }
  };
  if (rb < 1 || rb > 4 || rg < 0 || rg > 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bp_update<T>, dim3(L.n_update_items), dim3(kNT), 0, L.s, L.pairs,
                     L.npairs);
  box(true);
  hipLaunchKernelGGL(k_bp_decide, dim3(L.npairs), dim3(kNT), 0, L.s, L.pairs, dp);
  box(false);
  switch (rg) {
    case 0: launch_smooth_forms<0>(L); break;
    case 1: launch_smooth_forms<1>(L); break;
    case 2: launch_smooth_forms<2>(L); break;
    case 3: launch_smooth_forms<3>(L); break;
    case 4: launch_smooth_forms<4>(L); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_batch_phases(lmr_dtype t, lmr_accum accum, int box_radius,
                               int gauss_radius, bool march, bool bricks,
                               const BatchPair* pairs, int npairs, int n_update_items,
                               int n_tiles, const DecideParams& dp, hipStream_t s) {
  const PhaseLaunch L{pairs, npairs, n_update_items, n_tiles, march, bricks, s};
  if (accum == LMR_ACC_F32C)
    return t == LMR_BF16 ? phases_t<uint16_t, F32C>(L, box_radius, gauss_radius, dp)
                         : phases_t<float, F32C>(L, box_radius, gauss_radius, dp);
  return t == LMR_BF16 ? phases_t<uint16_t, double>(L, box_radius, gauss_radius, dp)
                       : phases_t<float, double>(L, box_radius, gauss_radius, dp);
}

}  // namespace lmr
