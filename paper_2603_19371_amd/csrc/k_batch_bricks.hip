// Batched persistent form, FP64 box sums, with 4-plane bricks for the pairs
// that run on them (a set of its own: it needs more registers).
#include "batch_attempt.h"

namespace lmr {

const void* batch_kernel_bricks(lmr_dtype t, int box_radius, int gauss_radius) {
  return batch_kernel_for<double, 1>(t, box_radius, gauss_radius);
}

}  // namespace lmr
