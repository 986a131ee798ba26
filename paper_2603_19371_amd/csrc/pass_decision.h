// The attempt's decision taken inside the backward pass (k_stencil.hip).
//
// On levels with few partial sums every block of the backward pass reduces
// them itself, in the fixed order of the decision kernel (decide.h), and takes
// the same decision, so the attempt needs no launch of its own for it: a
// rejected attempt's blocks return at once, block 0 stores the decided state
// in a staging slot, and the smoothing pass (always launched after it) makes
// that the pair state before it reads it.
#pragma once

#include "lmr_internal.h"

namespace lmr {

// Levels with at most this many partials take the decision in the backward
// pass; above it each block's reduction costs more than the launch it saves.
constexpr int kPassDecisionMaxParts = 1024;
// Box windows up to 2 * 3 + 1 = 7: with a wider window the deciding pass would
// spill registers at the occupancy of the pass without the decision.
constexpr int kPassDecisionMaxRadius = 3;

struct PassDecision {
  const double* partials;  // the forward pass's partials (null: no decision)
  int nparts;
  long long N;             // voxels: L = -sum / N
  DecideParams dp;
  int force;               // -1 the rule, 0/1 forced
  DevState* next;          // staging slot of the decided state (block 0 writes it)
  DevState* commit;        // smoothing pass: copy its state here first (or null)
};

// Whether the backward pass of this level takes the decision: at most
// kPassDecisionMaxParts partials, a window of at most 7, on the march or on
// 4-plane bricks (the 8-plane brick pass would spill registers with it).
bool bwd_takes_decision(const Geom& g, const lmr_params& p, int nparts);
// P4 with the decision: st is the pair state before the attempt (read only).
hipError_t launch_bwd_decide(const void* F, const void* M, lmr_dtype t, const float* Mw,
                             const float* maps, const Geom& g, const lmr_params& p,
                             const DevState* st, const float* U0, const float* U1,
                             const float* dMw, float* graw, const PassDecision& pd,
                             hipStream_t s);
// P5 after it: runs on the staged state `next` and stores it into the pair
// state st (block 0, before any block can return).
hipError_t launch_smooth_commit(const float* graw, const Geom& g, const lmr_params& p,
                                const DevState* next, DevState* st, float* out,
                                hipStream_t s);

}  // namespace lmr
