// Batched persistent form, FP64 box sums, marching pairs only; the dispatch
// over the instantiation sets and the launch.
#include "batch_attempt.h"

namespace lmr {

int batch_tile_rows() { return kTY; }
int batch_block_threads() { return kNT; }

const void* batch_kernel(lmr_dtype t, lmr_accum accum, int box_radius, int gauss_radius,
                         bool bricks) {
  if (accum == LMR_ACC_F32C)
    return bricks ? batch_kernel_bricks_f32c(t, box_radius, gauss_radius)
                  : batch_kernel_f32c(t, box_radius, gauss_radius);
  if (accum != LMR_ACC_F64) return nullptr;
  return bricks ? batch_kernel_bricks(t, box_radius, gauss_radius)
                : batch_kernel_for<double, 0>(t, box_radius, gauss_radius);
}

hipError_t launch_batch_attempt(const void* kernel, int grid, const BatchPair* pairs,
                                int npairs, int n_update_items, int n_tiles, BatchCtl* ctl,
                                const DecideParams& dp, unsigned long long timeout,
                                unsigned long long start_timeout, int missing,
                                hipStream_t s) {
  void* args[] = {&pairs,   &npairs,        &n_update_items, &n_tiles, &ctl,
                  const_cast<DecideParams*>(&dp), &timeout, &start_timeout, &missing};
  return hipLaunchKernel(kernel, dim3(grid), dim3(kNT), args, 0, s);
}

}  // namespace lmr
