// Coarse-to-fine pyramid (Sec. 2.1: each level inherits the warp of the
// previous one): average pooling of the images and x2 upsampling of the field.
//
//   k_avgpool        out = mean of each f^3 block, in FP32 whatever the input
//                    type (the pooled levels hold 1/8 or less of the voxels)
//   k_upsample_field fine index i samples the coarse field at (i - 0.5)/2,
//                    clamped to the coarse grid (voxel-centre alignment), by
//                    trilinear interpolation; the values are doubled because
//                    displacements are in voxels of the finer grid.
#include "pyramid.h"

namespace lmr {

namespace {

// FC > 0: the factor is FC, known at compile time, and the f^3 loads of an
// output are all requested before the first add (same order of additions);
// FC = 0: any factor f
template <typename T, int FC>
__global__ void __launch_bounds__(256)
    k_avgpool(const T* __restrict__ in, int nz, int ny, int nx, int f_rt,
              float* __restrict__ out) {
  const int f = FC > 0 ? FC : f_rt;
  const int cz = nz / f, cy = ny / f, cx = nx / f;
  const long long n = (long long)cz * cy * cx;
  const float inv = 1.0f / static_cast<float>(f * f * f);
  for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < n;
       o += (long long)gridDim.x * blockDim.x) {
    const int x = static_cast<int>(o % cx);
    const int y = static_cast<int>((o / cx) % cy);
    const int z = static_cast<int>(o / ((long long)cx * cy));
    float s = 0.0f;
    if constexpr (FC > 0) {
      float v[FC * FC * FC];
#pragma unroll
      for (int k = 0; k < FC; ++k)
#pragma unroll
        for (int j = 0; j < FC; ++j)
#pragma unroll
          for (int i = 0; i < FC; ++i)
            v[(k * FC + j) * FC + i] =
                ldf(in, ((long long)(z * FC + k) * ny + (y * FC + j)) * nx + (x * FC + i));
#pragma unroll
      for (int q = 0; q < FC * FC * FC; ++q) s += v[q];
    } else {
      for (int k = 0; k < f; ++k)
        for (int j = 0; j < f; ++j)
          for (int i = 0; i < f; ++i)
            s += ldf(in, ((long long)(z * f + k) * ny + (y * f + j)) * nx + (x * f + i));
    }
    out[o] = s * inv;
  }
}

__device__ __forceinline__ void src_coord(int i, int nc, int& i0, int& i1, float& t) {
  float s = (static_cast<float>(i) - 0.5f) * 0.5f;
  s = fminf(fmaxf(s, 0.0f), static_cast<float>(nc - 1));
  const float b = floorf(s);
  i0 = static_cast<int>(b);
  i1 = i0 + 1 < nc ? i0 + 1 : i0;
  t = s - b;
}

__global__ void __launch_bounds__(256)
    k_upsample_field(const DevState* __restrict__ st, const float* uc0,
                     const float* uc1, int nzc, int nyc, int nxc, float* __restrict__ uf) {
  // the coarse field: uc0, or with a pair state the buffer its ping-pong
  // index names (the level's current field, read where it lies)
  const float* __restrict__ uc = (st && st->cur) ? uc1 : uc0;
  const int nz = 2 * nzc, ny = 2 * nyc, nx = 2 * nxc;
  const long long N = (long long)nz * ny * nx, Nc = (long long)nzc * nyc * nxc;
  for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < N;
       o += (long long)gridDim.x * blockDim.x) {
    const int x = static_cast<int>(o % nx);
    const int y = static_cast<int>((o / nx) % ny);
    const int z = static_cast<int>(o / ((long long)nx * ny));
    int x0, x1, y0, y1, z0, z1;
    float tx, ty, tz;
    src_coord(x, nxc, x0, x1, tx);
    src_coord(y, nyc, y0, y1, ty);
    src_coord(z, nzc, z0, z1, tz);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* a = uc + c * Nc;
      auto at = [&](int zz, int yy, int xx) {
        return a[((long long)zz * nyc + yy) * nxc + xx];
      };
      const float v0 = (1 - ty) * ((1 - tx) * at(z0, y0, x0) + tx * at(z0, y0, x1)) +
                       ty * ((1 - tx) * at(z0, y1, x0) + tx * at(z0, y1, x1));
      const float v1 = (1 - ty) * ((1 - tx) * at(z1, y0, x0) + tx * at(z1, y0, x1)) +
                       ty * ((1 - tx) * at(z1, y1, x0) + tx * at(z1, y1, x1));
      uf[c * N + o] = 2.0f * ((1 - tz) * v0 + tz * v1);
    }
  }
}

unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace

hipError_t launch_avgpool(const void* in, lmr_dtype t, int nz, int ny, int nx, int f,
                          float* out, hipStream_t s) {
  const long long n = (long long)(nz / f) * (ny / f) * (nx / f);
  const dim3 grid(grid_for(n)), blk(256);
  if (t == LMR_BF16) {
    const auto* p = static_cast<const uint16_t*>(in);
    if (f == 2)
      hipLaunchKernelGGL((k_avgpool<uint16_t, 2>), grid, blk, 0, s, p, nz, ny, nx, f, out);
    else if (f == 4)
      hipLaunchKernelGGL((k_avgpool<uint16_t, 4>), grid, blk, 0, s, p, nz, ny, nx, f, out);
    else
      hipLaunchKernelGGL((k_avgpool<uint16_t, 0>), grid, blk, 0, s, p, nz, ny, nx, f, out);
  } else {
    const auto* p = static_cast<const float*>(in);
    if (f == 2)
      hipLaunchKernelGGL((k_avgpool<float, 2>), grid, blk, 0, s, p, nz, ny, nx, f, out);
    else if (f == 4)
      hipLaunchKernelGGL((k_avgpool<float, 4>), grid, blk, 0, s, p, nz, ny, nx, f, out);
    else
      hipLaunchKernelGGL((k_avgpool<float, 0>), grid, blk, 0, s, p, nz, ny, nx, f, out);
  }
  return hipGetLastError();
}

hipError_t launch_upsample_field(const float* uc, int nzc, int nyc, int nxc, float* uf,
                                 hipStream_t s) {
  return launch_upsample_cur(nullptr, uc, uc, nzc, nyc, nxc, uf, s);
}

hipError_t launch_upsample_cur(const DevState* st, const float* U0, const float* U1,
                               int nzc, int nyc, int nxc, float* uf, hipStream_t s) {
  const long long n = 8LL * nzc * nyc * nxc;
  hipLaunchKernelGGL(k_upsample_field, dim3(grid_for(n)), dim3(256), 0, s, st, U0, U1, nzc,
                     nyc, nxc, uf);
  return hipGetLastError();
}

}  // namespace lmr
