// Internal structures of the batched persistent form (k_batch.hip, api_batch.cpp).
#pragma once

#include "lmr_internal.h"
#include "stencil.h"

namespace lmr {

// One pair of a batch as the persistent kernel sees it (device memory).
struct BatchPair {
  Geom g;
  const void* F;
  const void* M;
  float* U0;
  float* U1;
  float* G;
  float* graw;
  float* maps;
  float* Mw;
  const double* fstat;  // window mean and variance of F (the pair context's)
  double* partials;  // one slot per stencil tile of this pair
  DevState* st;
  Tiling t;          // stencil tiling of this pair (marching form)
  int bricks;        // 1: the stencil work items are kBatchBrickTZ x 8 x 8 bricks
  int ntiles;        // stencil work items (and cc partials) of this pair
  int utile0;        // first update work item of this pair
  int ucz;           // planes per update work item of this pair
  int tile0;         // first stencil work item of this pair
  float eps;
  int compositive;
  double inv_n, cc_eps;
  float gw[16];      // Gaussian taps, 2R+1 <= 9 used
};

// Grid-barrier state and the timeout flag of the persistent kernel.  Blocks
// arrive on one of kBarGroups group counters (block id modulo the group
// count, one cache line each); the last arrival of a group arrives on the top
// counter, and the last of those releases everyone by raising the number of
// completed barriers `gen`, which lives on its own line so that the waiting
// blocks' polls do not contend with the arrivals.  The counters only grow
// (64 bits, never reset inside a kernel) and are touched by atomic
// read-modify-writes only: a block learns from its own arrival which barrier
// it is at, and no plain store to a counter has to be ordered against the
// atomics of blocks on other chiplets.
constexpr int kBarGroups = 8;
// Depth of the bricks of the pairs the batched kernel runs on bricks: those
// a stand-alone context also runs on 4-plane bricks (brick_depth), so that
// such a pair's run is the stand-alone run bit for bit.
constexpr int kBatchBrickTZ = 4;
// update work item: a 32 x 8 column (the staged update's tile) over ucz
// planes: about kBatchUpdateItems items per pair, 2..32 planes each (long
// marches for large pairs, short ones where a pair has few columns)
constexpr int kBatchUpdateTX = 32, kBatchUpdateTY = 8, kBatchUpdateItems = 256;
constexpr int kBatchUpdateMinCz = 2, kBatchUpdateMaxCz = 32;
struct BatchCtl {
  struct alignas(128) Line {
    unsigned long long v;
  };
  Line group[kBarGroups];
  Line top;
  Line gen;
  Line started[kBarGroups];  // blocks that have started (per group, as the
                             // arrivals), over all launches since the reset
  Line error;    // 1: a barrier wait timed out, 2: the grid was not co-resident
};

int batch_tile_rows();
int batch_block_threads();
// The persistent kernel for (image type, box-sum accumulator, box radius
// 1..4, Gaussian radius 0..4, whether some pair runs on bricks), or null when
// that combination is not instantiated.
const void* batch_kernel(lmr_dtype t, lmr_accum accum, int box_radius, int gauss_radius,
                         bool bricks);
// the sets of the above: compensated FP32 (k_batch_f32c.hip), with bricks
// (k_batch_bricks.hip, k_batch_bricks_f32c.hip)
const void* batch_kernel_f32c(lmr_dtype t, int box_radius, int gauss_radius);
const void* batch_kernel_bricks(lmr_dtype t, int box_radius, int gauss_radius);
const void* batch_kernel_bricks_f32c(lmr_dtype t, int box_radius, int gauss_radius);
// One attempt of every pair as one launch per phase (no persistent kernel):
// update, forward, decision, backward, smoothing; the stencil phases once
// for the marching pairs and once for the brick pairs, as present.
hipError_t launch_batch_phases(lmr_dtype t, lmr_accum accum, int box_radius,
                               int gauss_radius, bool march, bool bricks,
                               const BatchPair* pairs, int npairs, int n_update_items,
                               int n_tiles, const DecideParams& dp, hipStream_t s);
// timeout: ticks of a barrier wait; start_timeout: ticks after which a
// block waiting at the first barrier of a launch gives up if some block of
// the grid has not started; missing: 0, or 1 to make block 0 of every launch
// start 2 start_timeout late (exercises the co-residency failure).
hipError_t launch_batch_attempt(const void* kernel, int grid, const BatchPair* pairs,
                                int npairs, int n_update_items, int n_tiles, BatchCtl* ctl,
                                const DecideParams& dp, unsigned long long timeout,
                                unsigned long long start_timeout, int missing,
                                hipStream_t s);

}  // namespace lmr
