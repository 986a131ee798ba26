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
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

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
// Eight BF16 operand slots from two groups of four (bit patterns).
__device__ __forceinline__ b8 cat_bf16(s4 lo, s4 hi) {
  typedef short s8 __attribute__((ext_vector_type(8)));
  const s8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(b8, v);
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
// 16 x 16 (x, y) tile of output voxels in one z plane and 16 NT output
// channels; per chunk of 16 input channels it stages the 3 x 18 x 18 input
// halo and the chunk's 27 weight slices, then each wave runs the MFMAs of
// four 16-voxel rows for all 27 taps from LDS: each weight operand serves
// the four rows, each input operand the NT output-channel tiles.  Every load
// of a chunk is issued before the first is used (one memory latency per
// chunk, not one per load), and the next chunk's loads are in flight while
// the current chunk's MFMAs run.  Input positions outside the volume, and
// channels past cin_valid, read 0 through the buffer resource (an offset
// beyond the tensor).  (The streamed form above reads both operands from
// memory for every MFMA and is bound by the memory unit's per-instruction
// cost.)
//
// The MFMA computes D[co][voxel] = sum_ci W[co][ci] X[voxel][ci] (weights as
// the A operand), so that each lane receives four consecutive output channels
// of one voxel: the epilogue stores them as one 8-byte (BF16) or 16-byte
// (FP32) write.
//
// LDS rows (one voxel, or one weight row: 16 channels) are 40 bytes apart.
// An operand read takes the same 8-byte quad of 16 consecutive rows; with a
// 32-byte pitch those fall on 4 bank groups (a 4-way conflict), with 40
// bytes (10 dwords) 10 m mod 32 covers all 16 even banks.  The pitch keeps
// every LDS address affine in the tap, so the unrolled taps read at
// immediate offsets from one base per lane.
//
// Staging is arranged so that every address is a per-thread base plus a
// compile-time or per-block constant: the input halo is 54 rows (3 planes x
// 18 rows) of 72 items (18 voxels x 4 quads); threads 0..215 each take one
// item position in rows r0, r0 + 3, ... (r0 = thread / 72), 18 loads.
constexpr int kCT = 16;            // tile edge (x and y)
constexpr int kCH = kCT + 2;       // halo tile edge
constexpr int kPitch = 20;         // LDS row pitch, uint16 elements (40 bytes)
constexpr int kXLoads = 18;        // halo loads per staging thread
constexpr int kXThreads = 216;     // staging threads (3 rows x 72 items)
template <int NT>
__global__ void __launch_bounds__(256) k_conv_tile(ConvArgs a) {
  constexpr int kWRows = 27 * 16 * NT;            // weight rows per chunk
  constexpr int kWPer = (kWRows * 4 + 255) / 256;  // weight loads per thread
  constexpr int kTStep = 64 / (16 * NT);           // taps between a thread's loads
  __shared__ __attribute__((aligned(16))) uint16_t s_x[3 * kCH * kCH * kPitch];
  __shared__ __attribute__((aligned(16))) uint16_t s_w[kWRows * kPitch];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nco = a.cout_p / (16 * NT);
  // tile id: channel tile fastest, then x, y, z; each XCD takes a contiguous
  // range of ids, so the blocks that read an input plane (those of output
  // planes z-1, z, z+1, and every channel tile) mostly share one L2
  const int tiles_x = (a.nx + kCT - 1) / kCT, tiles_y = (a.ny + kCT - 1) / kCT;
  int b = xcd_remap(blockIdx.x, gridDim.x);
  const int co0 = (b % nco) * 16 * NT;
  b /= nco;
  const int x0 = (b % tiles_x) * kCT;
  b /= tiles_x;
  const int y0 = (b % tiles_y) * kCT;
  const int z = b / tiles_y;
  const int m = lane & 15, kq = lane >> 4;
  const int q = tid & 3;  // the quad (4 channels) this thread stages
  // ---- input staging: element offsets of this thread's 18 items (chunk 0)
  const long long nvox = (long long)a.nz * a.ny * a.nx;
  const RBuf bx = make_rbuf(
      a.X, static_cast<unsigned>(((nvox - 1) * a.ldx + ((a.cin_valid + 3) & ~3)) * 2));
  const int r0 = tid / 72, xx = (tid % 72) >> 2;
  const int gx = x0 + xx - 1;
  const bool xok = tid < kXThreads && (unsigned)gx < (unsigned)a.nx;
  const int row_st = a.nx * a.ldx, plane_st = a.ny * row_st;  // elements
  // item (zz, yi): voxel (gx, y0 + r0 + 3 yi - 1, z + zz - 1)
  const int xbase = ((z - 1) * a.ny + y0 + r0 - 1) * row_st + gx * a.ldx + 4 * q;
  unsigned yok = 0;  // bit yi: row y0 + r0 + 3 yi - 1 inside the volume
#pragma unroll
  for (int yi = 0; yi < 6; ++yi)
    yok |= ((unsigned)(y0 + r0 + 3 * yi - 1) < (unsigned)a.ny ? 1u : 0u) << yi;
  const int sx_base = (r0 * kCH + xx) * kPitch + 4 * q;  // LDS element offset
  // ---- weight staging: rows R = tid / 4 + 64 j (tap R / 16 NT, channel R % 16 NT)
  const RBuf bw = make_rbuf(a.W, static_cast<unsigned>(27LL * a.cout_p * a.cin_p * 2));
  const int wrow = tid >> 2;
  const int wbase = ((wrow / (16 * NT)) * a.cout_p + co0 + wrow % (16 * NT)) * a.cin_p + 4 * q;
  const int wstep = kTStep * a.cout_p * a.cin_p;
  s4 rx[kXLoads], rw[kWPer];
  auto fetch = [&](int c0) {
    const bool cok = xok && c0 + 4 * q < a.cin_valid;
#pragma unroll
    for (int i = 0; i < kXLoads; ++i) {
      const int zz = i / 6, yi = i % 6;
      const bool ok = cok && ((yok >> yi) & 1u) && (unsigned)(z + zz - 1) < (unsigned)a.nz;
      const int e = xbase + zz * plane_st + 3 * yi * row_st + c0;
      const unsigned o = ok ? static_cast<unsigned>(e) * 2u : kFarOffset;
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(bx.r, o, 0, 0);
      rx[i] = s4{static_cast<short>(v[0] & 0xFFFFu), static_cast<short>(v[0] >> 16),
                 static_cast<short>(v[1] & 0xFFFFu), static_cast<short>(v[1] >> 16)};
    }
#pragma unroll
    for (int j = 0; j < kWPer; ++j) {
      const unsigned o = wrow + 64 * j < kWRows
                             ? static_cast<unsigned>(wbase + j * wstep + c0) * 2u
                             : kFarOffset;
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(bw.r, o, 0, 0);
      rw[j] = s4{static_cast<short>(v[0] & 0xFFFFu), static_cast<short>(v[0] >> 16),
                 static_cast<short>(v[1] & 0xFFFFu), static_cast<short>(v[1] >> 16)};
    }
  };
  auto commit = [&]() {
    if (tid < kXThreads) {
#pragma unroll
      for (int i = 0; i < kXLoads; ++i)
        *reinterpret_cast<s4*>(&s_x[sx_base + i * 3 * kCH * kPitch]) = rx[i];
    }
#pragma unroll
    for (int j = 0; j < kWPer; ++j)
      if (wrow + 64 * j < kWRows)
        *reinterpret_cast<s4*>(&s_w[(wrow + 64 * j) * kPitch + 4 * q]) = rw[j];
  };
  f4 acc[NT][4];
#pragma unroll
  for (int n = 0; n < NT; ++n)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[n][r] = f4{0.f, 0.f, 0.f, 0.f};
  // operand bases: halo voxel (m, 4 wv) of plane 0, weight row m of tap 0
  const int xr_base = (4 * wv * kCH + m) * kPitch + 4 * kq;
  const int wr_base = m * kPitch + 4 * kq;
  fetch(0);
  for (int c0 = 0; c0 < a.cin_p; c0 += 16) {
    __syncthreads();  // the previous chunk's operands are no longer read
    commit();
    __syncthreads();
    if (c0 + 16 < a.cin_p) fetch(c0 + 16);  // in flight during this chunk's MFMAs
#pragma unroll 1
    for (int dz = 0; dz < 3; ++dz) {
      const uint16_t* xp = s_x + xr_base + dz * kCH * kCH * kPitch;
      const uint16_t* wp = s_w + wr_base + dz * 9 * 16 * NT * kPitch;
      // taps 2p and 2p + 1 as one K = 32 product (each lane's eight K slots:
      // its four channels of the first tap, then the same four of the
      // second, in both operands); the ninth tap as a K = 16 product
#pragma unroll
      for (int tp = 0; tp < 4; ++tp) {
        const int ta = 2 * tp, tb = ta + 1;
        b8 w[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n)
          w[n] = cat_bf16(*reinterpret_cast<const s4*>(wp + (ta * NT + n) * 16 * kPitch),
                          *reinterpret_cast<const s4*>(wp + (tb * NT + n) * 16 * kPitch));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const b8 xv = cat_bf16(
              *reinterpret_cast<const s4*>(xp + ((r + ta / 3) * kCH + ta % 3) * kPitch),
              *reinterpret_cast<const s4*>(xp + ((r + tb / 3) * kCH + tb % 3) * kPitch));
#pragma unroll
          for (int n = 0; n < NT; ++n)
            acc[n][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[n], xv, acc[n][r], 0, 0, 0);
        }
      }
      {
        constexpr int t9 = 8, dy = 2, dx = 2;  // halo coordinates of the ninth tap
        s4 w[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n)
          w[n] = *reinterpret_cast<const s4*>(wp + (t9 * NT + n) * 16 * kPitch);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const s4 xv = *reinterpret_cast<const s4*>(xp + ((r + dy) * kCH + dx) * kPitch);
#pragma unroll
          for (int n = 0; n < NT; ++n)
            acc[n][r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[n], xv, acc[n][r], 0, 0, 0);
        }
      }
    }
  }
  // D[4 kq + j][m]: output channel co0 + 16 n + 4 kq + j of voxel x0 + m in
  // row y0 + 4 wv + r
  const int x = x0 + m;
  if (x >= a.nx) return;
  const bool vec = a.cout % 4 == 0 && a.ldy % 4 == 0 && a.ldf % 4 == 0 &&
                   (reinterpret_cast<uintptr_t>(a.Y) % 8) == 0 &&
                   (reinterpret_cast<uintptr_t>(a.yf) % 16) == 0;
  // voxel of row r: v0 + r nx (v0: this lane's voxel in row y0 + 4 wv)
  const long long v0 = (long long)(z * a.ny + y0 + wv * 4) * a.nx + x;
  uint16_t* const yrow = a.Y ? a.Y + v0 * a.ldy : nullptr;
  float* const frow = a.yf ? a.yf + v0 * a.ldf : nullptr;
  const long long ystep = (long long)a.nx * a.ldy, fstep = (long long)a.nx * a.ldf;
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int cb = co0 + 16 * n + 4 * kq;
    if (cb >= a.cout) continue;
    float bias[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias[j] = (a.bias && cb + j < a.cout) ? a.bias[cb + j] : 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (y0 + wv * 4 + r >= a.ny) continue;
      float o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        o[j] = acc[n][r][j] + bias[j];
        if (a.relu) o[j] = fmaxf(o[j], 0.0f);
      }
      if (vec) {
        if (yrow) {
          const bf2 lo = __builtin_convertvector(f2{o[0], o[1]}, bf2);
          const bf2 hi = __builtin_convertvector(f2{o[2], o[3]}, bf2);
          *reinterpret_cast<uint2*>(yrow + r * ystep + cb) =
              uint2{__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)};
        }
        if (frow) *reinterpret_cast<f4*>(frow + r * fstep + cb) = f4{o[0], o[1], o[2], o[3]};
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (cb + j >= a.cout) continue;
          if (yrow) yrow[r * ystep + cb + j] = f2bf(o[j]);
          if (frow) frow[r * fstep + cb + j] = o[j];
        }
      }
    }
  }
}

// Weight gradient, partial over a brick of 16 x 16 (x, y) voxels and a range
// of z planes.  A block of four waves takes one brick, one tile of 16 input
// channels and one tile of 16 output channels; it marches through its planes
// with the input planes z-1, z, z+1 (halo 18 x 18) and the output-gradient
// plane z staged in LDS channel-major, so that a lane reads the four voxels
// of its K slots for one channel at once:
//   A[ci][k] = X[voxel k shifted by tap][ci],  B[k][co] = dZ[voxel k][co]
// with K running over 16 voxels of a row (lane group g takes voxels 4g..4g+3).
// Wave w owns rows 4w..4w+3 of the brick and keeps the 27 tap tiles in
// registers.  For one (dz, dy) a lane reads 6 consecutive halo voxels, which
// hold the operands of the three x taps (the shift by one voxel is a 16-bit
// funnel shift of the dwords).  The next planes' loads are in flight during
// the MFMAs of the current one.  At the end the four waves' tiles are added
// in LDS in wave order (a fixed order) and the block writes one partial;
// blocks of input tile 0 also sum dZ for the bias gradient.
constexpr int kWgPX = 20;   // X^T row pitch (elements): 18 halo voxels + pad (40 bytes)
constexpr int kWgPD = 20;   // dZ^T row pitch (elements): 16 voxels + pad (40 bytes)
constexpr int kWgXItems = kCH * kCH * 4;          // 8-byte items per input plane
constexpr int kWgXPer = (kWgXItems + 255) / 256;  // per thread
constexpr int kWgDPer = 16 * 16 * 4 / 256;        // dZ items per thread
constexpr int kWgSlot = kCH * 16 * kWgPX;         // elements per staged input plane
struct WgradArgs {
  const uint16_t* X;
  int ldx, cin, cin_p;
  const uint16_t* dZ;
  int ldz, cout, cout_p;
  int nz, ny, nx;
  int zper, nzp;  // planes per block, z parts
  float* part;
  float* partb;
};
__global__ void __launch_bounds__(256, 2) k_wgrad(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t s_xt[3 * kWgSlot];  // [slot][hy][ci][hx]
  __shared__ __attribute__((aligned(16))) uint16_t s_dt[16 * 16 * kWgPD];  // [y][co][x]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = lane & 15, kq = lane >> 4, q = tid & 3;
  const int nci = a.cin_p / 16, nco = a.cout_p / 16;
  const int nbx = (a.nx + 15) / 16, nby = (a.ny + 15) / 16;
  int b = blockIdx.x;
  const int cb = b % nco;
  b /= nco;
  const int ib = b % nci;
  b /= nci;
  const int chunk = b;  // (z part, brick y, brick x), brick x fastest
  const int bx = b % nbx;
  b /= nbx;
  const int by = b % nby;
  const int zp = b / nby;
  const int x0 = bx * 16, y0 = by * 16;
  const int zb = zp * a.zper, ze = min(a.nz, zb + a.zper);
  const long long nvox = (long long)a.nz * a.ny * a.nx;
  const RBuf rx = make_rbuf(
      a.X, static_cast<unsigned>(((nvox - 1) * a.ldx + ((a.cin + 3) & ~3)) * 2));
  const RBuf rd = make_rbuf(
      a.dZ, static_cast<unsigned>(((nvox - 1) * a.ldz + ((a.cout + 3) & ~3)) * 2));
  // input items of this thread: element offset within a plane (-1: reads 0)
  // and LDS position (without the slot and channel-in-quad terms)
  int xoff[kWgXPer], xl[kWgXPer];
  const bool cin_ok = ib * 16 + 4 * q < a.cin;
#pragma unroll
  for (int j = 0; j < kWgXPer; ++j) {
    const int it = tid + 256 * j;
    const int p = it >> 2, hy = p / kCH, hx = p % kCH;
    const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
    const bool ok = it < kWgXItems && cin_ok && (unsigned)gy < (unsigned)a.ny &&
                    (unsigned)gx < (unsigned)a.nx;
    xoff[j] = ok ? (gy * a.nx + gx) * a.ldx + ib * 16 + 4 * q : -1;
    xl[j] = it < kWgXItems ? (hy * 16 + 4 * q) * kWgPX + hx : -1;
  }
  // output-gradient items: voxel (x0 + dx_, y0 + dy_) with dy_ = tid / 64 + 4 j
  const int dx_ = (tid >> 2) & 15;
  const bool dcol_ok = x0 + dx_ < a.nx && cb * 16 + 4 * q < a.cout;
  const long long plane_x = (long long)a.ny * a.nx * a.ldx;
  uint2 px[kWgXPer], pd[kWgDPer];
  auto fetch_x = [&](int gz) {
    const bool zok = (unsigned)gz < (unsigned)a.nz;
#pragma unroll
    for (int j = 0; j < kWgXPer; ++j) {
      const unsigned o = zok && xoff[j] >= 0
                             ? static_cast<unsigned>((gz * plane_x + xoff[j]) * 2)
                             : kFarOffset;
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(rx.r, o, 0, 0);
      px[j] = uint2{static_cast<unsigned>(v[0]), static_cast<unsigned>(v[1])};
    }
  };
  auto fetch_d = [&](int gz) {
#pragma unroll
    for (int j = 0; j < kWgDPer; ++j) {
      const int gy = y0 + (tid >> 6) + 4 * j;
      const bool ok = dcol_ok && gy < a.ny;
      const long long e =
          ((long long)(gz * a.ny + gy) * a.nx + x0 + dx_) * a.ldz + cb * 16 + 4 * q;
      const unsigned o = ok ? static_cast<unsigned>(e * 2) : kFarOffset;
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(rd.r, o, 0, 0);
      pd[j] = uint2{static_cast<unsigned>(v[0]), static_cast<unsigned>(v[1])};
    }
  };
  // channel-major commits: 4 channels of one voxel go to 4 LDS rows
  auto commit_x = [&](int slot) {
    uint16_t* base = s_xt + slot * kWgSlot;
#pragma unroll
    for (int j = 0; j < kWgXPer; ++j) {
      if (xl[j] < 0) continue;
      uint16_t* d = base + xl[j];
      d[0] = static_cast<uint16_t>(px[j].x);
      d[kWgPX] = static_cast<uint16_t>(px[j].x >> 16);
      d[2 * kWgPX] = static_cast<uint16_t>(px[j].y);
      d[3 * kWgPX] = static_cast<uint16_t>(px[j].y >> 16);
    }
  };
  auto commit_d = [&]() {
#pragma unroll
    for (int j = 0; j < kWgDPer; ++j) {
      uint16_t* d = s_dt + (((tid >> 6) + 4 * j) * 16 + 4 * q) * kWgPD + dx_;
      d[0] = static_cast<uint16_t>(pd[j].x);
      d[kWgPD] = static_cast<uint16_t>(pd[j].x >> 16);
      d[2 * kWgPD] = static_cast<uint16_t>(pd[j].y);
      d[3 * kWgPD] = static_cast<uint16_t>(pd[j].y >> 16);
    }
  };
  f4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
  float bs = 0.0f;
  // planes zb - 1 and zb, then the march
  fetch_x(zb - 1);
  commit_x((zb + 2) % 3);
  fetch_x(zb);
  commit_x(zb % 3);
  fetch_x(zb + 1);
  fetch_d(zb);
  for (int z = zb; z < ze; ++z) {
    __syncthreads();  // the plane z - 2 slot and the dZ plane are no longer read
    commit_x((z + 1) % 3);
    commit_d();
    __syncthreads();
    if (z + 1 < ze) {
      fetch_x(z + 2);
      fetch_d(z + 1);
    }
    const uint16_t* xs[3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) xs[dz] = s_xt + ((z + 2 + dz) % 3) * kWgSlot;
    // rows 2p and 2p + 1 as one K = 32 product: each lane's eight K slots
    // are its four voxels of the first row, then the same four of the second
#pragma unroll
    for (int rp = 0; rp < 2; ++rp) {
      const int yl = 4 * wv + 2 * rp;
      const s4 bv0 = *reinterpret_cast<const s4*>(&s_dt[(yl * 16 + m) * kWgPD + 4 * kq]);
      const s4 bv1 = *reinterpret_cast<const s4*>(&s_dt[((yl + 1) * 16 + m) * kWgPD + 4 * kq]);
      if (ib == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) bs += bf2f(static_cast<uint16_t>(bv0[i]));
#pragma unroll
        for (int i = 0; i < 4; ++i) bs += bf2f(static_cast<uint16_t>(bv1[i]));
      }
      const b8 bv = cat_bf16(bv0, bv1);
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          // halo voxels 4 kq .. 4 kq + 5 of rows yl + dy and yl + 1 + dy,
          // channel m; the three x taps are one-voxel shifts of them
          s4 op[2][3];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const uint16_t* p = xs[dz] + ((yl + h + dy) * 16 + m) * kWgPX + 4 * kq;
            const uint2 w01 = *reinterpret_cast<const uint2*>(p);
            const unsigned w2 = *reinterpret_cast<const unsigned*>(p + 4);
            const unsigned a0 = __builtin_amdgcn_alignbit(w01.y, w01.x, 16);
            const unsigned a1 = __builtin_amdgcn_alignbit(w2, w01.y, 16);
            op[h][0] = __builtin_bit_cast(s4, uint2{w01.x, w01.y});  // dx = -1
            op[h][1] = __builtin_bit_cast(s4, uint2{a0, a1});        // dx = 0
            op[h][2] = __builtin_bit_cast(s4, uint2{w01.y, w2});     // dx = +1
          }
          const int t = dz * 9 + dy * 3;
#pragma unroll
          for (int d = 0; d < 3; ++d)
            acc[t + d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cat_bf16(op[0][d], op[1][d]),
                                                                 bv, acc[t + d], 0, 0, 0);
        }
    }
  }
  // the four waves' tiles added in LDS in wave order: D[4 kq + j][m] is
  // (input channel 4 kq + j, output channel m)
  float* red = reinterpret_cast<float*>(s_xt);  // 27 x 16 x 16 floats
  __shared__ float red_b[16];
  bs += __shfl_xor(bs, 16);
  bs += __shfl_xor(bs, 32);
  for (int w = 0; w < 4; ++w) {
    __syncthreads();
    if (wv == w) {
#pragma unroll
      for (int t = 0; t < 27; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float* d = red + (t * 16 + 4 * kq + j) * 16 + m;
          *d = (w == 0 ? 0.0f : *d) + acc[t][j];
        }
      if (kq == 0) red_b[m] = (w == 0 ? 0.0f : red_b[m]) + bs;
    }
  }
  __syncthreads();
  float* out = a.part + (long long)chunk * 27 * a.cin_p * a.cout_p;
  for (int e = tid; e < 27 * 256; e += 256) {
    const int t = e >> 8, ci = (e >> 4) & 15, co = e & 15;
    out[((long long)t * a.cin_p + ib * 16 + ci) * a.cout_p + cb * 16 + co] = red[e];
  }
  if (ib == 0 && tid < 16) a.partb[(long long)chunk * a.cout_p + cb * 16 + tid] = red_b[tid];
}

// dW[t][ci][co] = sum over chunks of the padded partials.  A block of 256
// threads reduces 16 consecutive outputs: 16 threads per output each sum the
// chunks c = q, q + 16, ... (q = the thread's share), then the 16 shares are
// added in order q = 0..15 (a fixed order, so the result does not depend on
// scheduling).  Many short sums in parallel instead of one long one per
// output: the partials of a layer can hold thousands of chunks.
constexpr int kRedShare = 16;
__global__ void __launch_bounds__(256)
    k_reduce_w(const float* __restrict__ part, int nchunks, int cin, int cout, int cin_p,
               int cout_p, float* __restrict__ dW, int accumulate) {
  __shared__ float red[kRedShare][256 / kRedShare];
  const long long n = 27LL * cin * cout, stride = 27LL * cin_p * cout_p;
  const int lo = threadIdx.x % (256 / kRedShare), q = threadIdx.x / (256 / kRedShare);
  const long long i = (long long)blockIdx.x * (256 / kRedShare) + lo;
  float s = 0.0f;
  if (i < n) {
    const int t = static_cast<int>(i / ((long long)cin * cout));
    const int r = static_cast<int>(i % ((long long)cin * cout));
    const long long o = ((long long)t * cin_p + r / cout) * cout_p + r % cout;
    for (int c = q; c < nchunks; c += kRedShare) s += part[c * stride + o];
  }
  red[q][lo] = s;
  __syncthreads();
  if (q == 0 && i < n) {
    float tot = 0.0f;
#pragma unroll
    for (int k = 0; k < kRedShare; ++k) tot += red[k][lo];
    dW[i] = accumulate ? dW[i] + tot : tot;
  }
}

__global__ void __launch_bounds__(256)
    k_reduce_b(const float* __restrict__ partb, int nchunks, int cout, int cout_p,
               float* __restrict__ db, int accumulate) {
  __shared__ float red[kRedShare][256 / kRedShare];
  const int lo = threadIdx.x % (256 / kRedShare), q = threadIdx.x / (256 / kRedShare);
  const int co = blockIdx.x * (256 / kRedShare) + lo;
  float s = 0.0f;
  if (co < cout)
    for (int c = q; c < nchunks; c += kRedShare) s += partb[(long long)c * cout_p + co];
  red[q][lo] = s;
  __syncthreads();
  if (q == 0 && co < cout) {
    float tot = 0.0f;
#pragma unroll
    for (int k = 0; k < kRedShare; ++k) tot += red[k][lo];
    db[co] = accumulate ? db[co] + tot : tot;
  }
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

// One block of 256 threads: thread t sums partials t, t + 256, ... in order,
// then a fixed tree adds the 256 sums (the result does not depend on timing).
__global__ void __launch_bounds__(256)
    k_mse_final(const double* __restrict__ part, int n, double inv, double* __restrict__ loss) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sh[0] * inv;
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

// Split of the weight gradient over z: about 512 blocks in total (two per
// compute unit), each marching through zper planes of one brick.
void wgrad_split(int cin_p, int cout_p, int nz, int ny, int nx, int& zper, int& nzp) {
  const long long per = (long long)(cin_p / 16) * (cout_p / 16) * ((nx + 15) / 16) *
                        ((ny + 15) / 16);
  long long want = (512 + per - 1) / per;
  if (want > nz) want = nz;
  if (want < 1) want = 1;
  zper = static_cast<int>((nz + want - 1) / want);
  nzp = (nz + zper - 1) / zper;
}
long long wgrad_chunks(int cin_p, int cout_p, int nz, int ny, int nx) {
  int zper, nzp;
  wgrad_split(cin_p, cout_p, nz, ny, nx, zper, nzp);
  return (long long)nzp * ((ny + 15) / 16) * ((nx + 15) / 16);
}

}  // namespace

hipError_t unet_conv(const ConvArgs& a, hipStream_t s) {
  const long long tile_bytes =
      ((long long)a.nz * a.ny * a.nx * a.ldx + ((a.cin_valid + 3) & ~3)) * 2;
  if (a.ldx % 4 == 0 && (reinterpret_cast<uintptr_t>(a.X) % 8) == 0 &&
      tile_bytes < static_cast<long long>(kFarOffset) - 16) {
    // 32 output channels per block where the layer has them: each input
    // operand read from LDS then feeds two MFMAs
    const int nt = a.cout_p % 32 == 0 ? 2 : 1;
    const long long nb = (long long)((a.nx + kCT - 1) / kCT) * ((a.ny + kCT - 1) / kCT) *
                         a.nz * (a.cout_p / (16 * nt));
    const dim3 grid(static_cast<unsigned>(nb));
    if (nt == 2)
      hipLaunchKernelGGL(k_conv_tile<2>, grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(k_conv_tile<1>, grid, dim3(256), 0, s, a);
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

long long unet_wgrad_part_floats(int cin_p, int cout_p, int nz, int ny, int nx) {
  return wgrad_chunks(cin_p, cout_p, nz, ny, nx) * 27 * cin_p * cout_p;
}

long long unet_wgrad_bias_floats(int cin_p, int cout_p, int nz, int ny, int nx) {
  return wgrad_chunks(cin_p, cout_p, nz, ny, nx) * cout_p;
}

hipError_t unet_wgrad(const uint16_t* X, int ldx, int cin, int cin_p, const uint16_t* dZ,
                      int ldz, int cout, int cout_p, int nz, int ny, int nx, float* part,
                      float* partb, float* dW, float* db, int accumulate, hipStream_t s) {
  // both tensors are read through 32-bit byte offsets
  const long long nvox = (long long)nz * ny * nx;
  if ((nvox * ldx + 4) * 2 >= static_cast<long long>(kFarOffset) ||
      (nvox * ldz + 4) * 2 >= static_cast<long long>(kFarOffset) || ldx % 4 || ldz % 4 ||
      reinterpret_cast<uintptr_t>(X) % 8 || reinterpret_cast<uintptr_t>(dZ) % 8)
    return hipErrorInvalidValue;
  WgradArgs w{X, ldx, cin, cin_p, dZ, ldz, cout, cout_p, nz, ny, nx, 0, 0, part, partb};
  wgrad_split(cin_p, cout_p, nz, ny, nx, w.zper, w.nzp);
  const long long nch = wgrad_chunks(cin_p, cout_p, nz, ny, nx);
  const unsigned blocks = static_cast<unsigned>(nch * (cin_p / 16) * (cout_p / 16));
  hipLaunchKernelGGL(k_wgrad, dim3(blocks), dim3(256), 0, s, w);
  const long long nw = 27LL * cin * cout, per = 256 / kRedShare;
  hipLaunchKernelGGL(k_reduce_w, dim3(static_cast<unsigned>((nw + per - 1) / per)), dim3(256),
                     0, s, part, static_cast<int>(nch), cin, cout, cin_p, cout_p, dW,
                     accumulate);
  hipLaunchKernelGGL(k_reduce_b, dim3(static_cast<unsigned>((cout + per - 1) / per)),
                     dim3(256), 0, s, partb, static_cast<int>(nch), cout, cout_p, db,
                     accumulate);
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
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, s, part, nb,
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
