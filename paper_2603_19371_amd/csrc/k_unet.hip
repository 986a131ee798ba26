// Kernels of the learned initializer's 3D U-Net: dense 3x3x3 convolutions
// on the MFMA matrix cores (BF16 operands, FP32 accumulation) and the
// memory-bound pieces around them (pooling, upsampling, ReLU gradient, MSE,
// Adam, weight packing).
//
// Layouts.  Activations are channels-last BF16: element (v, c) of a tensor
// with channel stride ld sits at v*ld + c, so a channel concatenation is two
// tensors sharing one buffer at different channel offsets.  Weights are FP32
// masters [27][cin][cout] (tap t = 9 (dz+1) + 3 (dy+1) + (dx+1) reads the
// input at v + (dx, dy, dz)), packed per step into BF16
//   Wf [27][cout_p][cin_p]  (forward: the reduction index contiguous)
//   Wb [27][cin_p][cout_p]  tap order reversed (gradient with respect to the
//                           input = convolution of dZ with the flipped,
//                           transposed kernel)
// with cin_p, cout_p the channel counts rounded up to 16, zero padded.
//
// MFMA operand layout (16x16 output tile, K = 4 g or 8 g per lane group
// g = lane / 16): lane l feeds row l % 16 of A and column l % 16 of B with
// the same K slots, and receives D[4 g + j][l % 16], j = 0..3.  Which K a
// slot maps to is irrelevant as long as A and B agree.
#include <hip/hip_runtime.h>

#include "lmr_internal.h"
#include "unet_internal.h"

namespace lmr {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t f2bf(float v) {
  uint32_t b = __float_as_uint(v);
  if ((b & 0x7F800000u) == 0x7F800000u)
    return static_cast<uint16_t>((b >> 16) | ((b & 0xFFFFu) ? 0x40u : 0u));
  b += 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// K = 16 per instruction: 4 BF16 per lane.
struct K16 {
  static constexpr int KW = 16;
  typedef s4 vec;
  __device__ static vec zero() { return vec{0, 0, 0, 0}; }
  __device__ static vec load(const uint16_t* p) { return *reinterpret_cast<const s4*>(p); }
  __device__ static f4 mma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};
// K = 32 per instruction (gfx950): 8 BF16 per lane.
struct K32 {
  static constexpr int KW = 32;
  typedef b8 vec;
  __device__ static vec zero() {
    vec z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = static_cast<__bf16>(0.0f);
    return z;
  }
  __device__ static vec load(const uint16_t* p) { return *reinterpret_cast<const b8*>(p); }
  __device__ static f4 mma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// ----------------------------------------------------------- convolution
// A block covers 64 consecutive output voxels along x (4 waves x 16) and 16
// output channels; K runs over the 27 taps and the input channels.
// A[m][k] = X[voxel x0 + m shifted by tap][channel], B[k][n] = W[tap][n][k].
template <class MM>
__global__ void __launch_bounds__(256) k_conv(ConvArgs a) {
  constexpr int KL = MM::KW / 4;  // K slots per lane
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x0 = blockIdx.x * 64 + wv * 16;
  if (x0 >= a.nx) return;
  const int nco = a.cout_p / 16;
  const int y = blockIdx.y;
  const int z = blockIdx.z / nco, co0 = (blockIdx.z % nco) * 16;
  const int m = lane & 15, kq = lane >> 4;
  const int xa = x0 + m;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int zz = z + dz, yy = y + dy, xx = xa + dx;
    const bool in = (unsigned)zz < (unsigned)a.nz && (unsigned)yy < (unsigned)a.ny &&
                    (unsigned)xx < (unsigned)a.nx;
    const uint16_t* xp =
        a.X + (in ? ((long long)(zz * a.ny + yy) * a.nx + xx) * a.ldx : 0);
    const uint16_t* wt = a.W + ((long long)t * a.cout_p + co0 + m) * a.cin_p;
    for (int c0 = 0; c0 < a.cin_p; c0 += MM::KW) {
      const int ci = c0 + KL * kq;
      typename MM::vec av = MM::zero();
      if (in && ci < a.cin_valid) av = MM::load(xp + ci);
      acc = MM::mma(av, MM::load(wt + ci), acc);
    }
  }
  const int co = co0 + m;
  if (co >= a.cout) return;
  const float b = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int xo = x0 + 4 * kq + j;
    if (xo >= a.nx) continue;
    const long long v = (long long)(z * a.ny + y) * a.nx + xo;
    float r = acc[j] + b;
    if (a.relu) r = fmaxf(r, 0.0f);
    if (a.Y) a.Y[v * a.ldy + co] = f2bf(r);
    if (a.yf) a.yf[v * a.ldf + co] = r;
  }
}

// The same convolution with the operands staged in LDS.  A block owns a
// 16 x 16 (x, y) tile of output voxels in one z plane and 16 output
// channels; per chunk of 16 input channels it stages the 3 x 18 x 18 input
// halo and the chunk's 27 weight slices, then each wave runs the MFMAs of
// four 16-voxel rows for all 27 taps from LDS, reusing each weight operand
// across its four rows.  (The streamed form above reads both operands from
// memory for every MFMA and is bound by the memory unit's per-instruction
// cost.)
constexpr int kCT = 16;            // tile edge (x and y)
constexpr int kCH = kCT + 2;       // halo tile edge
__global__ void __launch_bounds__(256) k_conv_tile(ConvArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t s_x[3][kCH][kCH][16];
  __shared__ __attribute__((aligned(16))) uint16_t s_w[27][16][16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nco = a.cout_p / 16;
  const int x0 = blockIdx.x * kCT, y0 = blockIdx.y * kCT;
  const int z = blockIdx.z / nco, co0 = (blockIdx.z % nco) * 16;
  const int m = lane & 15, kq = lane >> 4;
  f4 acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = f4{0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < a.cin_p; c0 += 16) {
    __syncthreads();  // the previous chunk's operands are no longer read
    // input halo: 3 x 18 x 18 voxels x 16 channels, 4 channels per item
    for (int it = threadIdx.x; it < 3 * kCH * kCH * 4; it += 256) {
      const int q = it & 3, p = it >> 2;
      const int xx = p % kCH, yy = (p / kCH) % kCH, zz = p / (kCH * kCH);
      const int gx = x0 + xx - 1, gy = y0 + yy - 1, gz = z + zz - 1;
      const int ci = c0 + 4 * q;
      s4 v = {0, 0, 0, 0};
      if ((unsigned)gx < (unsigned)a.nx && (unsigned)gy < (unsigned)a.ny &&
          (unsigned)gz < (unsigned)a.nz && ci < a.cin_valid)
        v = *reinterpret_cast<const s4*>(
            a.X + ((long long)(gz * a.ny + gy) * a.nx + gx) * a.ldx + ci);
      *reinterpret_cast<s4*>(&s_x[zz][yy][xx][4 * q]) = v;
    }
    // weights of the chunk: 27 taps x 16 output x 16 input channels
    for (int it = threadIdx.x; it < 27 * 16 * 4; it += 256) {
      const int q = it & 3, co = (it >> 2) & 15, t = it >> 6;
      *reinterpret_cast<s4*>(&s_w[t][co][4 * q]) = *reinterpret_cast<const s4*>(
          a.W + ((long long)t * a.cout_p + co0 + co) * a.cin_p + c0 + 4 * q);
    }
    __syncthreads();
#pragma unroll 3
    for (int t = 0; t < 27; ++t) {
      const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;  // halo coordinates
      const s4 b = *reinterpret_cast<const s4*>(&s_w[t][m][4 * kq]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int yl = wv * 4 + r;
        const s4 av = *reinterpret_cast<const s4*>(&s_x[dz][yl + dy][m + dx][4 * kq]);
        acc[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, b, acc[r], 0, 0, 0);
      }
    }
  }
  // D[4 kq + j][n]: voxel x0 + 4 kq + j of row y0 + 4 wv + r, output channel co0 + n
  const int co = co0 + m;
  if (co >= a.cout) return;
  const float bias = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int y = y0 + wv * 4 + r;
    if (y >= a.ny) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = x0 + 4 * kq + j;
      if (x >= a.nx) continue;
      const long long v = (long long)(z * a.ny + y) * a.nx + x;
      float o = acc[r][j] + bias;
      if (a.relu) o = fmaxf(o, 0.0f);
      if (a.Y) a.Y[v * a.ldy + co] = f2bf(o);
      if (a.yf) a.yf[v * a.ldf + co] = o;
    }
  }
}

// Weight gradient, partial over a chunk of (z, y) rows.  One wave per
// (chunk, 16 input channels, 16 output channels) keeps the 27 tap tiles in
// registers: A[m][k] = X[voxel k shifted by tap][ci m], B[k][n] = dZ[voxel k][co n]
// with K running over 16 voxels of a row.  The waves of input block 0 also
// sum dZ for the bias gradient.
__global__ void __launch_bounds__(64)
    k_wgrad(const uint16_t* __restrict__ X, int ldx, int cin, int cin_p,
            const uint16_t* __restrict__ dZ, int ldz, int cout, int cout_p, int nz, int ny,
            int nx, int rows_per_chunk, float* __restrict__ part,
            float* __restrict__ partb) {
  const int lane = threadIdx.x;
  const int nci = cin_p / 16, nco = cout_p / 16;
  int b = blockIdx.x;
  const int cb = b % nco;
  b /= nco;
  const int ib = b % nci;
  const int ch = b / nci;
  const int nrows = nz * ny;
  const int r0 = ch * rows_per_chunk, r1 = min(r0 + rows_per_chunk, nrows);
  const int m = lane & 15, kq = lane >> 4;
  const int ci = ib * 16 + m, co = cb * 16 + m;
  f4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
  float bs = 0.0f;
  for (int row = r0; row < r1; ++row) {
    const int z = row / ny, y = row % ny;
    for (int xb = 0; xb < nx; xb += 16) {
      s4 bb;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int x = xb + 4 * kq + j;
        bb[j] = (x < nx && co < cout)
                    ? static_cast<short>(dZ[((long long)row * nx + x) * ldz + co])
                    : static_cast<short>(0);
        bs += bf2f(static_cast<uint16_t>(bb[j]));
      }
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const int zz = z + dz, yy = y + dy;
        const bool rok = ci < cin && (unsigned)zz < (unsigned)nz && (unsigned)yy < (unsigned)ny;
        const uint16_t* xr = X + (rok ? (long long)(zz * ny + yy) * nx * ldx + ci : 0);
        s4 av;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int xx = xb + 4 * kq + j + dx;
          av[j] = (rok && (unsigned)xx < (unsigned)nx)
                      ? static_cast<short>(xr[(long long)xx * ldx])
                      : static_cast<short>(0);
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bb, acc[t], 0, 0, 0);
      }
    }
  }
  float* out = part + (long long)ch * 27 * cin_p * cout_p;
#pragma unroll
  for (int t = 0; t < 27; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      out[((long long)t * cin_p + ib * 16 + 4 * kq + j) * cout_p + cb * 16 + m] = acc[t][j];
  if (ib == 0) {
    bs += __shfl_xor(bs, 16);
    bs += __shfl_xor(bs, 32);
    if (kq == 0) partb[(long long)ch * cout_p + cb * 16 + m] = bs;
  }
}

// dW[t][ci][co] = sum over chunks (in chunk order) of the padded partials.
__global__ void k_reduce_w(const float* __restrict__ part, int nchunks, int cin, int cout,
                           int cin_p, int cout_p, float* __restrict__ dW, int accumulate) {
  const long long n = 27LL * cin * cout, stride = 27LL * cin_p * cout_p;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int t = static_cast<int>(i / ((long long)cin * cout));
    const int r = static_cast<int>(i % ((long long)cin * cout));
    const long long o = ((long long)t * cin_p + r / cout) * cout_p + r % cout;
    float s = 0.0f;
    for (int c = 0; c < nchunks; ++c) s += part[c * stride + o];
    dW[i] = accumulate ? dW[i] + s : s;
  }
}

__global__ void k_reduce_b(const float* __restrict__ partb, int nchunks, int cout,
                           int cout_p, float* __restrict__ db, int accumulate) {
  const int co = blockIdx.x * blockDim.x + threadIdx.x;
  if (co >= cout) return;
  float s = 0.0f;
  for (int c = 0; c < nchunks; ++c) s += partb[(long long)c * cout_p + co];
  db[co] = accumulate ? db[co] + s : s;
}

__global__ void k_relu_mask(uint16_t* __restrict__ d, int ldd, const uint16_t* __restrict__ a,
                            int lda, int C, long long N) {
  const long long n = N * C;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long v = i / C;
    const int c = static_cast<int>(i % C);
    if (!(bf2f(a[v * lda + c]) > 0.0f)) d[v * ldd + c] = 0;
  }
}

// ------------------------------------------------------- resampling ops
__device__ __forceinline__ long long child(int z, int y, int x, int k, int ny, int nx) {
  return ((long long)(2 * z + (k >> 2)) * ny + 2 * y + ((k >> 1) & 1)) * nx + 2 * x + (k & 1);
}

// 2x2x2 average pooling of C channels from fine dims (nz, ny, nx).
__global__ void k_pool2(const uint16_t* __restrict__ X, int ldx, int C, int nz, int ny,
                        int nx, uint16_t* __restrict__ Y, int ldy) {
  const int cy = ny / 2, cx = nx / 2;
  const long long n = (long long)(nz / 2) * cy * cx * C;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int c = static_cast<int>(i % C);
    const long long v = i / C;
    const int x = static_cast<int>(v % cx), y = static_cast<int>((v / cx) % cy),
              z = static_cast<int>(v / ((long long)cx * cy));
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += bf2f(X[child(z, y, x, k, ny, nx) * ldx + c]);
    Y[v * ldy + c] = f2bf(s * 0.125f);
  }
}

// Gradient of the pooling: every fine voxel receives dY / 8.
__global__ void k_pool2_back(const uint16_t* __restrict__ dY, int ldy, int C, int nz,
                             int ny, int nx, uint16_t* __restrict__ dX, int ldx, int add) {
  const long long n = (long long)nz * ny * nx * C;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int c = static_cast<int>(i % C);
    const long long v = i / C;
    const int x = static_cast<int>(v % nx), y = static_cast<int>((v / nx) % ny),
              z = static_cast<int>(v / ((long long)nx * ny));
    const long long cv = ((long long)(z / 2) * (ny / 2) + y / 2) * (nx / 2) + x / 2;
    float r = bf2f(dY[cv * ldy + c]) * 0.125f;
    if (add) r += bf2f(dX[v * ldx + c]);
    dX[v * ldx + c] = f2bf(r);
  }
}

// x2 nearest-neighbour upsampling to fine dims (nz, ny, nx).
__global__ void k_up2(const uint16_t* __restrict__ X, int ldx, int C, int nz, int ny,
                      int nx, uint16_t* __restrict__ Y, int ldy) {
  const long long n = (long long)nz * ny * nx * C;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int c = static_cast<int>(i % C);
    const long long v = i / C;
    const int x = static_cast<int>(v % nx), y = static_cast<int>((v / nx) % ny),
              z = static_cast<int>(v / ((long long)nx * ny));
    const long long cv = ((long long)(z / 2) * (ny / 2) + y / 2) * (nx / 2) + x / 2;
    Y[v * ldy + c] = X[cv * ldx + c];
  }
}

// The same, 8 channels per 16-byte access (C, strides and bases multiples of 8
// elements).
__global__ void k_up2_v8(const uint16_t* __restrict__ X, int ldx, int C, int nz, int ny,
                         int nx, uint16_t* __restrict__ Y, int ldy) {
  const int G = C / 8;
  const int n = nz * ny * nx * G;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int g = i % G, v = i / G;
    const int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
    const int cv = ((z >> 1) * (ny >> 1) + (y >> 1)) * (nx >> 1) + (x >> 1);
    *reinterpret_cast<uint4*>(Y + (long long)v * ldy + 8 * g) =
        *reinterpret_cast<const uint4*>(X + (long long)cv * ldx + 8 * g);
  }
}

// Gradient of the upsampling: the sum over the 8 fine children.
__global__ void k_up2_back(const uint16_t* __restrict__ dY, int ldy, int C, int nz, int ny,
                           int nx, uint16_t* __restrict__ dX, int ldx, int add) {
  const int cy = ny / 2, cx = nx / 2;
  const long long n = (long long)(nz / 2) * cy * cx * C;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int c = static_cast<int>(i % C);
    const long long v = i / C;
    const int x = static_cast<int>(v % cx), y = static_cast<int>((v / cx) % cy),
              z = static_cast<int>(v / ((long long)cx * cy));
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += bf2f(dY[child(z, y, x, k, ny, nx) * ldy + c]);
    if (add) s += bf2f(dX[v * ldx + c]);
    dX[v * ldx + c] = f2bf(s);
  }
}

template <typename T>
__global__ void k_input(const T* __restrict__ F, const T* __restrict__ M, int nz, int ny,
                        int nx, int pool, uint16_t* __restrict__ X) {
  const long long n = (long long)nz * ny * nx;
  const int fy = pool ? 2 * ny : ny, fx = pool ? 2 * nx : nx;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < n;
       v += (long long)gridDim.x * blockDim.x) {
    float f = 0.0f, m = 0.0f;
    if (pool) {
      const int x = static_cast<int>(v % nx), y = static_cast<int>((v / nx) % ny),
                z = static_cast<int>(v / ((long long)nx * ny));
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int i = static_cast<int>(child(z, y, x, k, fy, fx));
        f += ldf(F, i);
        m += ldf(M, i);
      }
      f *= 0.125f;
      m *= 0.125f;
    } else {
      f = ldf(F, static_cast<int>(v));
      m = ldf(M, static_cast<int>(v));
    }
    X[v * 4 + 0] = f2bf(f);
    X[v * 4 + 1] = f2bf(m);
    X[v * 4 + 2] = 0;
    X[v * 4 + 3] = 0;
  }
}

__global__ void k_head_to_field(const float* __restrict__ yf, int ldf, long long N,
                                float* __restrict__ field) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < 3; ++c) field[c * N + v] = yf[v * ldf + c];
}

// Squared error per block (FP64) and the BF16 gradient 2 (out - target) / (3N).
__global__ void __launch_bounds__(256)
    k_mse(const float* __restrict__ yf, int ldf, const float* __restrict__ target,
          float tscale, long long N, uint16_t* __restrict__ dout, int ld,
          double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  const float scale = static_cast<float>(2.0 / (3.0 * static_cast<double>(N)));
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float d = yf[v * ldf + c] - tscale * target[c * N + v];
      s += static_cast<double>(d) * d;
      dout[v * ld + c] = f2bf(scale * d);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mse_final(const double* __restrict__ part, int n, double inv,
                            double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *loss = s * inv;
}

__global__ void k_fill_u16(uint16_t* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Adam on FP32 master parameters (bias-corrected moments: c1 = 1 - b1^t,
// c2 = 1 - b2^t); the gradient is scaled by gscale first.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long long n, float lr, float b1,
                       float b2, float eps, float c1, float c2, float gscale) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i] * gscale;
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void k_pack(const float* __restrict__ W, int cin, int cout, int cin_p,
                       int cout_p, uint16_t* __restrict__ Wf, uint16_t* __restrict__ Wb) {
  const long long n = 27LL * cin_p * cout_p;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int t = static_cast<int>(i / ((long long)cin_p * cout_p));
    const int r = static_cast<int>(i % ((long long)cin_p * cout_p));
    const int ci = r / cout_p, co = r % cout_p;
    const float w = (ci < cin && co < cout) ? W[((long long)t * cin + ci) * cout + co] : 0.0f;
    const uint16_t h = f2bf(w);
    Wf[((long long)t * cout_p + co) * cin_p + ci] = h;
    Wb[((long long)(26 - t) * cin_p + ci) * cout_p + co] = h;
  }
}

unsigned grid_n(long long n) {
  long long b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

// Row chunking of the weight gradient: about 4096 waves in total.
void wgrad_chunks(int cin_p, int cout_p, int nz, int ny, int& nchunks, int& rpc) {
  const int nrows = nz * ny;
  const int per = (cin_p / 16) * (cout_p / 16);
  int want = (4096 + per - 1) / per;
  if (want > nrows) want = nrows;
  if (want < 1) want = 1;
  rpc = (nrows + want - 1) / want;
  nchunks = (nrows + rpc - 1) / rpc;
}

}  // namespace

hipError_t unet_conv(const ConvArgs& a, hipStream_t s) {
  if (a.ldx % 4 == 0 && (reinterpret_cast<uintptr_t>(a.X) % 8) == 0) {
    dim3 grid((a.nx + kCT - 1) / kCT, (a.ny + kCT - 1) / kCT, a.nz * (a.cout_p / 16));
    hipLaunchKernelGGL(k_conv_tile, grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  dim3 grid((a.nx + 63) / 64, a.ny, a.nz * (a.cout_p / 16));
  const bool k32 = a.cin_p % 32 == 0 && a.ldx % 8 == 0 && a.cin_valid % 8 == 0 &&
                   (reinterpret_cast<uintptr_t>(a.X) % 16) == 0;
  if (k32)
    hipLaunchKernelGGL(k_conv<K32>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_conv<K16>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

long long unet_wgrad_part_floats(int cin_p, int cout_p, int nz, int ny) {
  int nch, rpc;
  wgrad_chunks(cin_p, cout_p, nz, ny, nch, rpc);
  return (long long)nch * 27 * cin_p * cout_p;
}

long long unet_wgrad_bias_floats(int cin_p, int cout_p, int nz, int ny) {
  int nch, rpc;
  wgrad_chunks(cin_p, cout_p, nz, ny, nch, rpc);
  return (long long)nch * cout_p;
}

hipError_t unet_wgrad(const uint16_t* X, int ldx, int cin, int cin_p, const uint16_t* dZ,
                      int ldz, int cout, int cout_p, int nz, int ny, int nx, float* part,
                      float* partb, float* dW, float* db, int accumulate, hipStream_t s) {
  int nch, rpc;
  wgrad_chunks(cin_p, cout_p, nz, ny, nch, rpc);
  const unsigned blocks = static_cast<unsigned>(nch * (cin_p / 16) * (cout_p / 16));
  hipLaunchKernelGGL(k_wgrad, dim3(blocks), dim3(64), 0, s, X, ldx, cin, cin_p, dZ, ldz,
                     cout, cout_p, nz, ny, nx, rpc, part, partb);
  hipLaunchKernelGGL(k_reduce_w, dim3(grid_n(27LL * cin * cout)), dim3(256), 0, s, part,
                     nch, cin, cout, cin_p, cout_p, dW, accumulate);
  hipLaunchKernelGGL(k_reduce_b, dim3((cout + 127) / 128), dim3(128), 0, s, partb, nch,
                     cout, cout_p, db, accumulate);
  return hipGetLastError();
}

hipError_t unet_relu_mask(uint16_t* d, int ldd, const uint16_t* a, int lda, int C,
                          long long N, hipStream_t s) {
  hipLaunchKernelGGL(k_relu_mask, dim3(grid_n(N * C)), dim3(256), 0, s, d, ldd, a, lda, C, N);
  return hipGetLastError();
}

hipError_t unet_pool2(const uint16_t* X, int ldx, int C, int nz, int ny, int nx,
                      uint16_t* Y, int ldy, hipStream_t s) {
  hipLaunchKernelGGL(k_pool2, dim3(grid_n((long long)nz * ny * nx * C / 8)), dim3(256), 0,
                     s, X, ldx, C, nz, ny, nx, Y, ldy);
  return hipGetLastError();
}

hipError_t unet_pool2_back(const uint16_t* dY, int ldy, int C, int nz, int ny, int nx,
                           uint16_t* dX, int ldx, int add, hipStream_t s) {
  hipLaunchKernelGGL(k_pool2_back, dim3(grid_n((long long)nz * ny * nx * C)), dim3(256), 0,
                     s, dY, ldy, C, nz, ny, nx, dX, ldx, add);
  return hipGetLastError();
}

hipError_t unet_up2(const uint16_t* X, int ldx, int C, int nz, int ny, int nx, uint16_t* Y,
                    int ldy, hipStream_t s) {
  if (C % 8 == 0 && ldx % 8 == 0 && ldy % 8 == 0 &&
      reinterpret_cast<uintptr_t>(X) % 16 == 0 && reinterpret_cast<uintptr_t>(Y) % 16 == 0) {
    hipLaunchKernelGGL(k_up2_v8, dim3(grid_n((long long)nz * ny * nx * C / 8)), dim3(256),
                       0, s, X, ldx, C, nz, ny, nx, Y, ldy);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_up2, dim3(grid_n((long long)nz * ny * nx * C)), dim3(256), 0, s, X,
                     ldx, C, nz, ny, nx, Y, ldy);
  return hipGetLastError();
}

hipError_t unet_up2_back(const uint16_t* dY, int ldy, int C, int nz, int ny, int nx,
                         uint16_t* dX, int ldx, int add, hipStream_t s) {
  hipLaunchKernelGGL(k_up2_back, dim3(grid_n((long long)nz * ny * nx * C / 8)), dim3(256),
                     0, s, dY, ldy, C, nz, ny, nx, dX, ldx, add);
  return hipGetLastError();
}

hipError_t unet_input(const void* F, const void* M, lmr_dtype t, int nz, int ny, int nx,
                      int pool, uint16_t* X, hipStream_t s) {
  const long long n = (long long)nz * ny * nx;
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_input<uint16_t>, dim3(grid_n(n)), dim3(256), 0, s,
                       static_cast<const uint16_t*>(F), static_cast<const uint16_t*>(M), nz,
                       ny, nx, pool, X);
  else
    hipLaunchKernelGGL(k_input<float>, dim3(grid_n(n)), dim3(256), 0, s,
                       static_cast<const float*>(F), static_cast<const float*>(M), nz, ny,
                       nx, pool, X);
  return hipGetLastError();
}

hipError_t unet_head_to_field(const float* yf, int ldf, long long N, float* field,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_head_to_field, dim3(grid_n(N)), dim3(256), 0, s, yf, ldf, N, field);
  return hipGetLastError();
}

int unet_mse_blocks(long long N) {
  const unsigned g = grid_n(N);
  return static_cast<int>(g > 1024 ? 1024 : g);
}

hipError_t unet_mse(const float* yf, int ldf, const float* target, float tscale,
                    long long N, uint16_t* dout, int ld, double* part, double* loss,
                    hipStream_t s) {
  const int nb = unet_mse_blocks(N);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, yf, ldf, target, tscale, N, dout, ld,
                     part);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, s, part, nb,
                     1.0 / (3.0 * static_cast<double>(N)), loss);
  return hipGetLastError();
}

hipError_t unet_zero(uint16_t* p, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u16, dim3(grid_n(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t unet_adam(float* p, float* m, float* v, const float* g, long long n, float lr,
                     float b1, float b2, float eps, float c1, float c2, float gscale,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_n(n)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2,
                     eps, c1, c2, gscale);
  return hipGetLastError();
}

hipError_t unet_pack(const float* W, int cin, int cout, int cin_p, int cout_p,
                     uint16_t* Wf, uint16_t* Wb, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(grid_n(27LL * cin_p * cout_p)), dim3(256), 0, s, W, cin,
                     cout, cin_p, cout_p, Wf, Wb);
  return hipGetLastError();
}

}  // namespace lmr
