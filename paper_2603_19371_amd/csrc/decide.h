// The on-device decision of one LM attempt, as a block-wide device function
// shared by the per-pair decision kernel and the batched persistent kernel.
//
// The cc partial sums are reduced in a fixed order in FP64 into
// L = -sum cc / N; then (Sec. 2.2, eq. lambda-update; Sec. 3.4,
// eq. rejection):
//   reject iff L is not finite, or tau >= 0 and
//              L - L(t-1) > tau |L(t-1) - L(t-2)|   (reference 0 with < 2 losses)
//   accept:    lambda <- mu+ lambda if L > L(t-1) else mu- lambda, clamped;
//              the loss history shifts and the field ping-pong index flips
//   reject:    lambda <- min(mu+ lambda, lambda_max); after max_retries
//              consecutive rejections at lambda_max the pair is frozen.
#pragma once

#include "lmr_internal.h"

namespace lmr {

__device__ __forceinline__ double clamp_d(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// The sum of the partials in a fixed order, by all NT threads of one block
// (sh: NT doubles of LDS); the result is valid in thread 0.
template <int NT>
__device__ double reduce_partials(const double* __restrict__ partials, int nparts,
                                  double* sh) {
  static_assert(NT >= 64 && (NT & (NT - 1)) == 0, "power-of-two block of whole waves");
  // each thread sums partials t, t + NT, t + 2 NT, ... in that order; the
  // first kLoads of them are all requested before the first add, so a level
  // with up to kLoads * NT partials waits for one memory round trip, not one
  // per NT partials
  constexpr int kLoads = 8;
  double v[kLoads];
#pragma unroll
  for (int j = 0; j < kLoads; ++j) {
    const int k = threadIdx.x + j * NT;
    v[j] = k < nparts ? partials[k] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kLoads; ++j)
    if (threadIdx.x + j * NT < nparts) s += v[j];
  for (int k = threadIdx.x + kLoads * NT; k < nparts; k += NT) s += partials[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  // the fixed tree sh[t] += sh[t + w], w = NT/2 ... 1: the steps across waves
  // in LDS, the last six inside wave 0 with the same operands and order
  for (int w = NT / 2; w >= 64; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  double v0 = 0.0;
  if (threadIdx.x < 64) {
    v0 = sh[threadIdx.x];
#pragma unroll
    for (int w = 32; w > 0; w >>= 1) v0 += __shfl_down(v0, w, 64);
  }
  return v0;
}

// The state after an attempt whose candidate has loss L, from the state cur
// read before it (force -1: the rule; 0/1: a forced decision).  A frozen pair
// only records that nothing was accepted.
__device__ inline DevState decide_next(const DevState& cur, double L, const DecideParams& dp,
                                       int force) {
  DevState n = cur;
  if (cur.stalled) {
    n.accepted = 0;
    return n;
  }
  n.cand_loss = L;
  n.attempts += 1;
  int acc;
  if (force >= 0) {
    acc = force ? 1 : 0;
  } else if (!isfinite(L)) {
    acc = 0;
  } else if (dp.tau < 0.0) {
    acc = 1;
  } else {
    const double ref = n.n_hist >= 2 ? fabs(n.loss - n.loss_prev) : 0.0;
    acc = !((L - n.loss) > dp.tau * ref);
  }
  if (acc) {
    const double f = (L > n.loss) ? dp.lambda_inc : dp.lambda_dec;
    n.lambda = clamp_d(f * n.lambda, dp.lambda_min, dp.lambda_max);
    n.loss_prev = n.loss;
    n.loss = L;
    n.r = residual_of(L, dp.similarity, dp.mi_bins);
    n.n_hist += 1;
    n.retries = 0;
    n.cur = 1 - n.cur;
  } else {
    n.lambda = clamp_d(dp.lambda_inc * n.lambda, dp.lambda_min, dp.lambda_max);
    n.retries += 1;
    if (n.retries >= dp.max_retries && n.lambda >= dp.lambda_max) n.stalled = 1;
  }
  n.accepted = acc;
  // beta^t of the step that follows (t = attempts + 1)
  n.adam_pow1 *= dp.adam_beta1;
  n.adam_pow2 *= dp.adam_beta2;
  return n;
}

// mode 0: attempt (force -1/0/1), mode 1: begin (lambda0), mode 2: probe
// (*probe = L).  Called by all NT threads of one block; uses NT doubles of LDS.
template <int NT>
__device__ void decide_block(DevState* st, const double* __restrict__ partials,
                             int nparts, long long N, const DecideParams& dp, int mode,
                             int force, double lambda0, double* probe) {
  __shared__ double sh[NT];
  // thread 0 fetches the state while the partials are being loaded
  DevState cur_st;
  if (threadIdx.x == 0) cur_st = *st;
  const double S = reduce_partials<NT>(partials, nparts, sh);
  if (threadIdx.x == 0) {
    const double L = -S / static_cast<double>(N);
    if (mode == 2) {
      *probe = L;
    } else if (mode == 1) {
      st->lambda = lambda0;
      st->loss = L;
      st->loss_prev = L;
      st->cand_loss = L;
      st->r = residual_of(L, dp.similarity, dp.mi_bins);
      st->n_hist = 1;
      st->retries = 0;
      st->accepted = 1;
      st->stalled = 0;
      st->cur = 0;
      st->attempts = 0;
      st->adam_pow1 = dp.adam_beta1;
      st->adam_pow2 = dp.adam_beta2;
    } else {
      // the decision on the state read at entry; the new state is written back
      *st = decide_next(cur_st, L, dp, force);
    }
  }
  __syncthreads();
}

}  // namespace lmr
