// Batched persistent form, compensated FP32 box sums (LMR_ACC_F32C).
#include "batch_attempt.h"

namespace lmr {

const void* batch_kernel_f32c(lmr_dtype t, int box_radius, int gauss_radius) {
  return batch_kernel_for<F32C, 0>(t, box_radius, gauss_radius);
}

}  // namespace lmr
