// Separable 3D stencils of one LM attempt on a shared 2.5D framework, as
// device functions used by the per-pair kernels (k_stencil.hip) and by the
// batched persistent kernel (k_batch.hip).
//
//   FStatPol  window mean and variance of F, once per pair.
//   FwdPol    LNCC forward: box sums of Mw, Mw^2, F Mw over the w^3 window
//             (zero padding, divisor w^3), cc = s_FM^2/(s_FF s_MM + eps),
//             adjoint maps alpha = 2 s_FM/D, alpha mu_F, beta = -s_FM^2 s_FF/D^2,
//             beta mu_M, and one FP64 partial sum of cc per tile.
//   BwdPol    LNCC backward: box sums of the four maps give
//             d(sum cc)/dMw_j = (F_j B(alpha) - B(alpha mu_F) + 2 Mw_j B(beta)
//                                - 2 B(beta mu_M)) / w^3,
//             times the trilinear derivative of M at x + u(x) (warp backward);
//             the result is g = N dL/du with L = -mean cc.
//   SmoothPol Gaussian of the raw gradient (Eulerian descent, Sec. 2.1).
//
// A tile is a 32 x TY column of outputs over a chunk of z planes.  For each
// input plane the block stages a (TY+2R) x (32+2R) halo tile of the raw FP32
// inputs in LDS (the next plane is already in flight in registers while the
// current one is reduced), reduces along y (expanding the raw inputs into the
// accumulated channels: for the forward pass the exact products F^2, Mw^2,
// F Mw in FP64) and then along x, and keeps the last 2R+1 plane sums in a
// register ring.  Box sums run a running sum through the ring; the Gaussian
// sums it with its taps.
#pragma once

#include <type_traits>

#include "lmr_internal.h"

namespace lmr {

constexpr int kTX = 32;

// Compensated FP32 accumulator (the LMR_ACC_F32C box sums): an unevaluated
// sum hi + lo of two floats, accumulated by cascaded summation.  The high
// parts add with Knuth's TwoSum, whose exact rounding error joins the low
// parts, which add plainly; a product of two floats enters exactly through
// the FMA remainder.  No renormalisation between additions.  The y- and
// x-passes take 2R+1 additions each; the running z-sum of a tile takes two
// per plane of its march (the entering plane and the leaving one), i.e.
// 2 (cz + 2R) of them, about 200 on a 96-plane chunk.  Every TwoSum error is
// at most half an ulp of the running hi, so after k additions |lo| is at
// most about k/2 ulp(hi), and the plain additions of lo add an error of at
// most k^2/4 * 2^-24 ulp(hi): below 0.01 ulp(hi) for k = 200.  hi + lo
// therefore keeps about twice FP32's significand over a whole chunk.  With
// contraction off the sequences run as written.
struct F32C {
  float hi, lo;
  F32C() = default;  // trivial, so LDS arrays may hold it; F32C() value-initialises to 0
  __host__ __device__ explicit F32C(float v) : hi(v), lo(0.0f) {}
  __device__ static F32C product(float a, float b) {
    F32C r{};
    r.hi = a * b;
    r.lo = fmaf(a, b, -r.hi);
    return r;
  }
  __device__ friend F32C operator+(const F32C& a, const F32C& b) {
    F32C r{};
    r.hi = a.hi + b.hi;
    const float bb = r.hi - a.hi;
    const float e = (a.hi - (r.hi - bb)) + (b.hi - bb);
    r.lo = (a.lo + b.lo) + e;
    return r;
  }
  __device__ friend F32C operator-(const F32C& a, const F32C& b) {
    F32C nb{};
    nb.hi = -b.hi;
    nb.lo = -b.lo;
    return a + nb;
  }
  __device__ F32C& operator+=(const F32C& b) { return *this = *this + b; }
};
__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(const F32C& v) {
  return static_cast<double>(v.hi) + static_cast<double>(v.lo);
}

struct Tiling {
  int ty, tiles_x, tiles_y, nchunks, cz;
  __host__ __device__ int tiles() const { return tiles_x * tiles_y * nchunks; }
};

constexpr int kMinTiles = 256;  // one tile per CU

// Floor on the chunk length: 8 planes while that still gives every CU a tile
// (the 2R halo planes stay a moderate share), else 4, else 2 when 4 would
// leave CUs without a tile (small pyramid levels: the march of a chunk is
// their latency).
__host__ __device__ inline int march_floor_cz(long long cols, int nz) {
  return cols * ((nz + 7) / 8) >= kMinTiles   ? 8
         : cols * ((nz + 3) / 4) >= kMinTiles ? 4
                                              : 2;
}

// z-chunk: long enough that the 2R halo planes of a chunk stay a small
// fraction when the volume is large, short enough that small volumes still
// give a few hundred tiles.  target_tiles and min_cz are tuning knobs.
__host__ __device__ inline Tiling make_tiling(int nz, int ny, int nx, int ty,
                                              int target_tiles = 2048, int min_cz = 16) {
  Tiling t;
  t.ty = ty;
  t.tiles_x = (nx + kTX - 1) / kTX;
  t.tiles_y = (ny + ty - 1) / ty;
  const int cols = t.tiles_x * t.tiles_y;
  const int want = (target_tiles + cols - 1) / cols;
  int cz = (nz + want - 1) / want;
  if (cols * ((nz + min_cz - 1) / min_cz) >= target_tiles / 2 && cz < min_cz) cz = min_cz;
  const int floor_cz = march_floor_cz(cols, nz);
  if (cz < floor_cz) cz = floor_cz;
  if (cz > nz) cz = nz;
  t.cz = cz;
  t.nchunks = (nz + cz - 1) / cz;
  return t;
}

// The depth of the bricks the stencil passes of a stand-alone context run on
// (4 or 8 planes), or 0 where they march (k_stencil.hip); and the number of
// bricks of depth tz.
int brick_depth(const Geom& g, const lmr_params& p);
int brick_count(const Geom& g, int tz);

// The march's tiling of a volume for stencil radius R on the current device
// (k_stencil.hip): every pass of a per-pair attempt, and by default each pair
// of the batched form.
Tiling march_tiling(const Geom& g, int R);

// LDS of one stencil tile: the staged raw inputs and the y-pass sums.
template <int R, int TY, class P>
struct StencilLds {
  float in[P::NRAW][TY + 2 * R][kTX + 2 * R];
  typename P::Acc y[P::NCH][TY][kTX + 2 * R];
};

// Runs the stencil over tile (x0, y0, z0..z1) with the whole block, in the
// LDS arrays s_in (staged raw inputs) and s_y (y-pass sums).
template <int R, int TY, class P>
__device__ __forceinline__ void stencil_tile_in(
    const P& pol, const Geom& g, int x0, int y0, int z0, int z1, typename P::Local& loc,
    float (&s_in)[P::NRAW][TY + 2 * R][kTX + 2 * R],
    typename P::Acc (&s_y)[P::NCH][TY][kTX + 2 * R]) {
  using A = typename P::Acc;
  constexpr int NR = P::NRAW, NC = P::NCH;
  constexpr int W = 2 * R + 1, LX = kTX + 2 * R, LY = TY + 2 * R, NT = kTX * TY;
  constexpr int NPOS = LX * LY, PER = (NPOS + NT - 1) / NT;

  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool own = gx < g.nx && gy < g.ny;
  const int plane = g.ny * g.nx;

  // positions of the halo tile this thread stages
  int pidx[PER];
  bool pin[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int i = threadIdx.x + p * NT;
    const int yy = i / LX, xx = i - yy * LX;
    const int gyy = y0 - R + yy, gxx = x0 - R + xx;
    pin[p] = i < NPOS && (unsigned)gyy < (unsigned)g.ny && (unsigned)gxx < (unsigned)g.nx;
    pidx[p] = pin[p] ? gyy * g.nx + gxx : 0;
  }
  // Branch-free staging: a padding position (outside the volume in x, y or z)
  // reads kFarIndex, whose offset lies beyond the buffer and reads 0.
  float pre[PER][NR];
  auto fetch = [&](int zi) {
    const bool zin = (unsigned)zi < (unsigned)g.nz;
    const unsigned zoff = zin ? static_cast<unsigned>(zi * plane) : 0u;
#pragma unroll
    for (int p = 0; p < PER; ++p)
      pol.load(loc, (zin && pin[p]) ? zoff + static_cast<unsigned>(pidx[p]) : kFarIndex,
               pre[p]);
  };
  auto commit = [&]() {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int i = threadIdx.x + p * NT;
      if (i < NPOS) {
        const int yy = i / LX, xx = i - yy * LX;
#pragma unroll
        for (int c = 0; c < NR; ++c) s_in[c][yy][xx] = pre[p][c];
      }
    }
  };

  A ring[W][NC], run[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    run[c] = A();
#pragma unroll
    for (int k = 0; k < W; ++k) ring[k][c] = A();
  }

  const int zend = z1 + R;
  int zi = z0 - R;
  fetch(zi);
  while (zi < zend) {
#pragma unroll
    for (int s = 0; s < W; ++s) {
      if (zi < zend) {
        commit();
        if (zi + 1 < zend) fetch(zi + 1);
        __syncthreads();
        for (int i = threadIdx.x; i < TY * LX; i += NT) {
          const int yy = i / LX, xx = i - yy * LX;
          A a[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) a[c] = A();
#pragma unroll
          for (int k = 0; k < W; ++k) {
            float r[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) r[c] = s_in[c][yy + k][xx];
            pol.accum(a, r, k);
          }
#pragma unroll
          for (int c = 0; c < NC; ++c) s_y[c][yy][xx] = a[c];
        }
        __syncthreads();
        A pl[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) pl[c] = A();
#pragma unroll
        for (int k = 0; k < W; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            if constexpr (P::kBox)
              pl[c] += s_y[c][ly][lx + k];
            else
              pl[c] = fma(A(pol.wt(k)), s_y[c][ly][lx + k], pl[c]);
          }
        A sm[NC];
        if constexpr (P::kBox) {
          // ring[s] holds the plane that entered W steps ago
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            run[c] += pl[c] - ring[s][c];
            ring[s][c] = pl[c];
            sm[c] = run[c];
          }
        } else {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            ring[s][c] = pl[c];
            sm[c] = A(0);
          }
          // planes zi-2R .. zi sit in slots s+1 .. s+W (mod W)
#pragma unroll
          for (int k = 0; k < W; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c)
              sm[c] = fma(A(pol.wt(k)), ring[(s + 1 + k) % W][c], sm[c]);
        }
        const int zo = zi - R;
        if (zo >= z0 && own) pol.emit(loc, zo * plane + gy * g.nx + gx, gx, gy, zo, sm);
      }
      ++zi;
    }
  }
}

// In the LDS `sm` (a kernel that runs several phases overlays their LDS).
template <int R, int TY, class P>
__device__ __forceinline__ void stencil_tile(const P& pol, const Geom& g, int x0, int y0,
                                             int z0, int z1, typename P::Local& loc,
                                             StencilLds<R, TY, P>& sm) {
  stencil_tile_in<R, TY>(pol, g, x0, y0, z0, z1, loc, sm.in, sm.y);
}

// In LDS of its own.  Both forms give the same results; the compiler
// schedules them differently, and the backward pass runs faster with two
// separate arrays, the others with one struct (measured).
template <int R, int TY, class P>
__device__ __forceinline__ void stencil_tile(const P& pol, const Geom& g, int x0, int y0,
                                             int z0, int z1, typename P::Local& loc) {
  if constexpr (P::kSeparateLds) {
    __shared__ float s_in[P::NRAW][TY + 2 * R][kTX + 2 * R];
    __shared__ typename P::Acc s_y[P::NCH][TY][kTX + 2 * R];
    stencil_tile_in<R, TY>(pol, g, x0, y0, z0, z1, loc, s_in, s_y);
  } else {
    __shared__ StencilLds<R, TY, P> sm;
    stencil_tile_in<R, TY>(pol, g, x0, y0, z0, z1, loc, sm.in, sm.y);
  }
}

// ------------------------------------------------------------- 3D tiles
// Small volumes (coarse pyramid levels) have too few 32 x TY columns to fill
// the GPU, and the plane-serial march of a short chunk is their latency.
// There a block owns a whole TZ x kT3 x kT3 brick of outputs instead: each
// thread reads one (y, x) column of the (kT3 + 2R)^2 halo straight from
// memory (all its loads in flight at once) and reduces along z, expanding the
// raw inputs into the accumulated channels; then the block reduces along y
// and along x in LDS and emits.  Three steps instead of a march.
constexpr int kT3 = 8;
constexpr int kCubeThreads = 256;

// The z sums of the halo columns.  The y pass reads them, keeps its own
// (fewer) results in registers and, after a barrier, writes them over the z
// sums, so one array serves both passes and more blocks fit on a CU.
template <int R, class P, int TZ>
struct CubeLds {
  using A = typename P::Acc;
  static constexpr int L = kT3 + 2 * R;
  A z[P::NCH][TZ][L][L];
  __device__ __forceinline__ A (&y())[P::NCH][TZ][kT3][L] {
    return *reinterpret_cast<A(*)[P::NCH][TZ][kT3][L]>(&z[0][0][0][0]);
  }
};

template <int R, int TZ, class P>
__device__ __forceinline__ void stencil_cube(const P& pol, const Geom& g, int x0, int y0,
                                             int z0, typename P::Local& loc,
                                             CubeLds<R, P, TZ>& sm) {
  using A = typename P::Acc;
  constexpr int NR = P::NRAW, NC = P::NCH, W = 2 * R + 1, L = kT3 + 2 * R;
  constexpr int NT = kCubeThreads;
  // z: one (y, x) column of the halo per thread
  for (int col = threadIdx.x; col < L * L; col += NT) {
    const int yy = col / L, xx = col - yy * L;
    const int gy = y0 - R + yy, gx = x0 - R + xx;
    const bool in = (unsigned)gy < (unsigned)g.ny && (unsigned)gx < (unsigned)g.nx;
    float r[TZ + 2 * R][NR];
#pragma unroll
    for (int k = 0; k < TZ + 2 * R; ++k) {
      const int gz = z0 - R + k;
      const unsigned i = (in && (unsigned)gz < (unsigned)g.nz)
                             ? static_cast<unsigned>((gz * g.ny + gy) * g.nx + gx)
                             : kFarIndex;
      pol.load(loc, i, r[k]);
    }
    if constexpr (P::kBox) {
      // running sum down the column: the entering position's terms are
      // added, the leaving position's (formed again) subtracted
      A a[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) a[c] = A();
#pragma unroll
      for (int k = 0; k < W; ++k) pol.accum(a, r[k], k);
#pragma unroll
      for (int oz = 0; oz < TZ; ++oz) {
#pragma unroll
        for (int c = 0; c < NC; ++c) sm.z[c][oz][yy][xx] = a[c];
        if (oz + 1 < TZ) {
          A in_[NC], out_[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) in_[c] = out_[c] = A();
          pol.accum(in_, r[oz + W], 0);
          pol.accum(out_, r[oz], 0);
#pragma unroll
          for (int c = 0; c < NC; ++c) a[c] += in_[c] - out_[c];
        }
      }
    } else {
#pragma unroll
      for (int oz = 0; oz < TZ; ++oz) {
        A a[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) a[c] = A();
#pragma unroll
        for (int k = 0; k < W; ++k) pol.accum(a, r[oz + k], k);
#pragma unroll
        for (int c = 0; c < NC; ++c) sm.z[c][oz][yy][xx] = a[c];
      }
    }
  }
  __syncthreads();
  // y, into registers first
  constexpr int NY = TZ * kT3 * L, KY = (NY + NT - 1) / NT;
  A ay[KY][NC];
#pragma unroll
  for (int j = 0; j < KY; ++j) {
    const int it = threadIdx.x + j * NT;
    if (NY % NT == 0 || it < NY) {
      const int oz = it / (kT3 * L), rem = it - oz * (kT3 * L);
      const int oy = rem / L, xx = rem - oy * L;
#pragma unroll
      for (int c = 0; c < NC; ++c) ay[j][c] = A();
#pragma unroll
      for (int k = 0; k < W; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if constexpr (P::kBox)
            ay[j][c] += sm.z[c][oz][oy + k][xx];
          else
            ay[j][c] = fma(A(pol.wt(k)), sm.z[c][oz][oy + k][xx], ay[j][c]);
        }
    }
  }
  __syncthreads();
  auto& sy = sm.y();
#pragma unroll
  for (int j = 0; j < KY; ++j) {
    const int it = threadIdx.x + j * NT;
    if (NY % NT == 0 || it < NY) {
      const int oz = it / (kT3 * L), rem = it - oz * (kT3 * L);
      const int oy = rem / L, xx = rem - oy * L;
#pragma unroll
      for (int c = 0; c < NC; ++c) sy[c][oz][oy][xx] = ay[j][c];
    }
  }
  __syncthreads();
  // x, and the outputs
  for (int it = threadIdx.x; it < TZ * kT3 * kT3; it += NT) {
    const int oz = it / (kT3 * kT3), oy = (it / kT3) % kT3, ox = it % kT3;
    A a[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) a[c] = A();
#pragma unroll
    for (int k = 0; k < W; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if constexpr (P::kBox)
          a[c] += sy[c][oz][oy][ox + k];
        else
          a[c] = fma(A(pol.wt(k)), sy[c][oz][oy][ox + k], a[c]);
      }
    const int gx = x0 + ox, gy = y0 + oy, gz = z0 + oz;
    if (gx < g.nx && gy < g.ny && gz < g.nz)
      pol.emit(loc, (gz * g.ny + gy) * g.nx + gx, gx, gy, gz, a);
  }
}

// Block sum of one double per thread; thread 0 writes it to *out.
template <int NT>
__device__ __forceinline__ void block_sum_to(double v, double* out) {
  __shared__ double red[NT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) s += red[k];
    *out = s;
  }
  __syncthreads();
}

// ------------------------------------------------- statistics of F (once)
// The window mean and variance of the fixed image do not change between
// attempts: they are box-summed once per pair (at begin) and stored in FP64
// as mu_F and sigma_FF, from sums of the exact products F^2.
template <typename T, typename AccT = double>
struct FStatPol {
  using Acc = AccT;
  static constexpr int NRAW = 1, NCH = 2;
  static constexpr bool kBox = true, kSeparateLds = false;
  const T* __restrict__ F;
  double* __restrict__ fstat;  // [2][N]: mu_F, sigma_FF
  int N;
  double inv_n;
  struct Local {
    RBuf bF;
  };

  __device__ static constexpr double wt(int) { return 1.0; }
  __device__ Local begin_block(const DevState*) const { return Local{make_rbuf_n(F, N)}; }
  __device__ void load(const Local& l, unsigned i, float v[1]) const { v[0] = bld<T>(l.bF, i); }
  __device__ void accum(Acc a[2], const float r[1], int) const {
    if constexpr (std::is_same<Acc, F32C>::value) {
      a[0] += F32C(r[0]);
      a[1] += F32C::product(r[0], r[0]);
    } else {
      const double f = r[0];
      a[0] += f;
      a[1] = fma(f, f, a[1]);
    }
  }
  __device__ void emit(Local&, int i, int, int, int, const Acc S[2]) const {
    const double muF = to_f64(S[0]) * inv_n;
    fstat[i] = muF;
    fstat[N + i] = to_f64(S[1]) * inv_n - muF * muF;
  }
  __device__ void end_tile(Local&, int) const {}
};

// ------------------------------------------------------------- forward (P2)
// Box sums of Mw, Mw^2 and F Mw (exact products in FP64); mu_F and sigma_FF
// come from FStatPol's pass over the same F.
template <typename T, int NT, typename AccT = double>
struct FwdPol {
  using Acc = AccT;
  static constexpr int NRAW = 2, NCH = 3;
  static constexpr bool kBox = true, kSeparateLds = false;
  const T* __restrict__ F;
  const float* __restrict__ Mw;
  const double* __restrict__ fstat;
  float* __restrict__ maps;
  float* __restrict__ cc;
  double* __restrict__ partials;
  int N;
  double inv_n, eps;
  struct Local {
    double sum;
    RBuf bF, bM;
  };

  __device__ static constexpr double wt(int) { return 1.0; }
  __device__ Local begin_block(const DevState*) const {
    return Local{0.0, make_rbuf_n(F, N), make_rbuf_n(Mw, N)};
  }
  __device__ void load(const Local& l, unsigned i, float v[2]) const {
    v[0] = bld<T>(l.bF, i);
    v[1] = bld<float>(l.bM, i);
  }
  __device__ void accum(Acc a[3], const float r[2], int) const {
    if constexpr (std::is_same<Acc, F32C>::value) {
      a[0] += F32C(r[1]);
      a[1] += F32C::product(r[1], r[1]);
      a[2] += F32C::product(r[0], r[1]);
    } else {
      const double f = r[0], m = r[1];
      a[0] += m;
      a[1] = fma(m, m, a[1]);
      a[2] = fma(f, m, a[2]);
    }
  }
  __device__ void emit(Local& loc, int i, int, int, int, const Acc S[3]) const {
    const double muF = fstat[i], sff = fstat[N + i];
    const double muM = to_f64(S[0]) * inv_n;
    const double sfm = to_f64(S[2]) * inv_n - muF * muM;
    const double smm = to_f64(S[1]) * inv_n - muM * muM;
    const double iD = 1.0 / (sff * smm + eps);
    const double c = sfm * sfm * iD;
    const double alpha = 2.0 * sfm * iD;
    const double beta = -c * sff * iD;
    maps[i] = static_cast<float>(alpha);
    maps[N + i] = static_cast<float>(alpha * muF);
    maps[2 * N + i] = static_cast<float>(beta);
    maps[3 * N + i] = static_cast<float>(beta * muM);
    if (cc) cc[i] = static_cast<float>(c);
    loc.sum += c;
  }
  // partial sum of cc of the tile just processed, to partials[slot]
  __device__ void end_tile(Local& loc, int slot) const {
    block_sum_to<NT>(loc.sum, partials + slot);
    loc.sum = 0.0;
  }
};

// ------------------------------------------------------------ backward (P4)
template <typename T, typename AccT = double>
struct BwdPol {
  using Acc = AccT;
  static constexpr int NRAW = 4, NCH = 4;
  static constexpr bool kBox = true, kSeparateLds = true;
  const T* __restrict__ F;
  const T* __restrict__ M;
  const float* __restrict__ Mw;
  const float* __restrict__ maps;
  const float* U0;  // field ping-pong (state mode: the field is U[cur])
  const float* U1;
  const float* u_explicit;  // the field when no state is given
  // derivative of M at x + u(x) as the update kernel stored it for the
  // candidate (null: gathered here); may alias graw (read, then overwritten,
  // by the thread of the same voxel)
  const float* dMw;
  float* graw;
  Geom g;
  double inv_n;
  struct Local {
    RBuf bmap[4];
    RBuf bM;
    const float* u;
  };

  __device__ static constexpr double wt(int) { return 1.0; }
  __device__ Local begin_block(const DevState* st) const {
    const int N = static_cast<int>(g.N);
    Local l;
    l.u = st ? (st->cur ? U1 : U0) : u_explicit;
#pragma unroll
    for (int c = 0; c < 4; ++c) l.bmap[c] = make_rbuf_n(maps + c * N, N);
    l.bM = make_rbuf_n(M, N);
    return l;
  }
  __device__ void load(const Local& l, unsigned i, float v[4]) const {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = bld<float>(l.bmap[c], i);
  }
  __device__ void accum(Acc a[4], const float r[4], int) const {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if constexpr (std::is_same<Acc, F32C>::value)
        a[c] += F32C(r[c]);
      else
        a[c] += static_cast<double>(r[c]);
    }
  }
  __device__ void emit(const Local& loc, int i, int x, int y, int z, const Acc Bs[4]) const {
    const int N = static_cast<int>(g.N);
    const float* u = loc.u;
    const double fj = ldf(F, i), mj = Mw[i];
    const double B[4] = {to_f64(Bs[0]), to_f64(Bs[1]), to_f64(Bs[2]), to_f64(Bs[3])};
    const double dS = (fj * B[0] - B[1] + 2.0 * mj * B[2] - 2.0 * B[3]) * inv_n;
    const float d = static_cast<float>(dS);
    float gm[3];
    if (dMw) {
      gm[0] = dMw[i];
      gm[1] = dMw[N + i];
      gm[2] = dMw[2 * N + i];
    } else {
      float v[8];
      const BCell c = make_bcell(g, x, y, z, u[i], u[N + i], u[2 * N + i]);
      bcorners<T>(loc.bM, g, c, v);
      binterp(c, v, gm);
    }
    graw[i] = -d * gm[0];
    graw[N + i] = -d * gm[1];
    graw[2 * N + i] = -d * gm[2];
  }
  __device__ void end_tile(Local&, int) const {}
};

// ----------------------------------------------------------- smoothing (P5)
template <int R>
struct SmoothPol {
  using Acc = float;
  static constexpr int NRAW = 3, NCH = 3;
  static constexpr bool kBox = false, kSeparateLds = false;
  const float* __restrict__ in;
  float* __restrict__ out;
  int N;
  float w[2 * R + 1];
  struct Local {
    RBuf b[3];
  };

  __device__ float wt(int k) const { return w[k]; }
  __device__ Local begin_block(const DevState*) const {
    return Local{{make_rbuf_n(in, N), make_rbuf_n(in + N, N), make_rbuf_n(in + 2 * N, N)}};
  }
  __device__ void load(const Local& l, unsigned i, float v[3]) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = bld<float>(l.b[c], i);
  }
  __device__ void accum(float a[3], const float r[3], int k) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) a[c] = fmaf(w[k], r[c], a[c]);
  }
  __device__ void emit(Local&, int i, int, int, int, const float S[3]) const {
    out[i] = S[0];
    out[N + i] = S[1];
    out[2 * N + i] = S[2];
  }
  __device__ void end_tile(Local&, int) const {}
};

// Normalised Gaussian taps k in [-R, R] (host side).
template <int R>
inline void gauss_taps(double sigma, float* w) {
  double t[2 * R + 1], tot = 0.0;
  for (int k = -R; k <= R; ++k) {
    t[k + R] = R == 0 ? 1.0 : exp(-(double)k * k / (2.0 * sigma * sigma));
    tot += t[k + R];
  }
  for (int k = 0; k <= 2 * R; ++k) w[k] = static_cast<float>(t[k] / tot);
}

// Decode a tile index (x fastest, then y, then z chunk).
__device__ __forceinline__ void tile_origin(const Tiling& t, int b, int ty, int& x0,
                                            int& y0, int& z0) {
  const int tx_i = b % t.tiles_x;
  const int ty_i = (b / t.tiles_x) % t.tiles_y;
  const int ch = b / (t.tiles_x * t.tiles_y);
  x0 = tx_i * kTX;
  y0 = ty_i * ty;
  z0 = ch * t.cz;
}

}  // namespace lmr
