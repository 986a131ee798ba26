// Level hand-off of the coarse-to-fine pyramid (k_pyramid.hip).
#pragma once

#include "lmr_internal.h"

namespace lmr {

// x2 upsampling of the coarse field into uf ([3][2nzc][2nyc][2nxc], values
// doubled), reading it from U1 if the pair state st (device) has its ping-pong
// index set, else from U0: the coarse level's current field, where it lies.
hipError_t launch_upsample_cur(const DevState* st, const float* U0, const float* U1,
                               int nzc, int nyc, int nxc, float* uf, hipStream_t s);

}  // namespace lmr
