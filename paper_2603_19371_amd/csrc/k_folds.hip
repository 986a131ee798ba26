// Folded-voxel count: voxels where det(I + grad u) <= 0.
//
// Partial derivatives are central differences inside the volume and
// first-order one-sided differences on its faces.  The determinant is
// expanded along the first row in FP64 with contraction into fused
// multiply-adds disabled, in the same operation order as a plain expansion
// on the host, so that the integer decision det <= 0 does not depend on
// rounding differences between implementations.
#include "lmr_internal.h"

namespace lmr {

namespace {

constexpr int kBX = 64, kBY = 4;

__device__ __forceinline__ double dcomp(const float* __restrict__ a, const Geom& g, int x,
                                        int y, int z, int axis) {
  const int n = axis == 0 ? g.nx : (axis == 1 ? g.ny : g.nz);
  const int i = axis == 0 ? x : (axis == 1 ? y : z);
  if (n < 2) return 0.0;
  const int lo = i > 0 ? i - 1 : i, hi = i < n - 1 ? i + 1 : i;
  int ilo, ihi;
  if (axis == 0) {
    ilo = (z * g.ny + y) * g.nx + lo;
    ihi = (z * g.ny + y) * g.nx + hi;
  } else if (axis == 1) {
    ilo = (z * g.ny + lo) * g.nx + x;
    ihi = (z * g.ny + hi) * g.nx + x;
  } else {
    ilo = (lo * g.ny + y) * g.nx + x;
    ihi = (hi * g.ny + y) * g.nx + x;
  }
  // hi - lo is 1 or 2, and x * 0.5 equals x / 2 exactly
  const double diff = static_cast<double>(a[ihi]) - static_cast<double>(a[ilo]);
  return hi - lo == 2 ? diff * 0.5 : diff;
}

__global__ void __launch_bounds__(kBX* kBY)
    k_folds(const float* __restrict__ u, Geom g, unsigned long long* __restrict__ count,
            float* __restrict__ det_out) {
#pragma clang fp contract(off)
  __shared__ unsigned red[kBX * kBY / 64];
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  unsigned folded = 0;
  if (x < g.nx && y < g.ny) {
    const int N = static_cast<int>(g.N);
    double J[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        J[c][d] = (c == d ? 1.0 : 0.0) + dcomp(u + c * N, g, x, y, z, d);
    const double D = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (det_out) det_out[(z * g.ny + y) * g.nx + x] = static_cast<float>(D);
    folded = D <= 0.0 ? 1u : 0u;
  }
  // wave count by ballot, then one integer atomic per block
  const int t = threadIdx.y * kBX + threadIdx.x;
  const unsigned wave = __popcll(__ballot(folded));
  if ((t & 63) == 0) red[t >> 6] = wave;
  __syncthreads();
  if (t == 0) {
    unsigned s = 0;
#pragma unroll
    for (int k = 0; k < kBX * kBY / 64; ++k) s += red[k];
    if (s) atomicAdd(count, static_cast<unsigned long long>(s));
  }
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

}  // namespace

hipError_t launch_folds(const float* u, const Geom& g, unsigned long long* count,
                        float* det, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, count);
  dim3 grid((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY, g.nz);
  hipLaunchKernelGGL(k_folds, grid, dim3(kBX, kBY), 0, s, u, g, count, det);
  return hipGetLastError();
}

}  // namespace lmr
