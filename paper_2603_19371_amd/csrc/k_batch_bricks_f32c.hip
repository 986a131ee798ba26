// Batched persistent form, compensated FP32 box sums, with 4-plane bricks for
// the pairs that run on them.
#include "batch_attempt.h"

namespace lmr {

const void* batch_kernel_bricks_f32c(lmr_dtype t, int box_radius, int gauss_radius) {
  return batch_kernel_for<F32C, 1>(t, box_radius, gauss_radius);
}

}  // namespace lmr
