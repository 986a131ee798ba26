// Separable 3D stencils of one LM attempt, on a shared 2.5D framework.
//
//   lncc_fwd  LNCC forward: box sums of F, Mw, F^2, Mw^2, F Mw over the w^3
//             window (zero padding, divisor w^3), cc = s_FM^2/(s_FF s_MM + eps),
//             adjoint maps alpha = 2 s_FM/D, alpha mu_F, beta = -s_FM^2 s_FF/D^2,
//             beta mu_M, and one FP64 partial sum of cc per block.
//   lncc_bwd  LNCC backward: box sums of the four maps give
//             d(sum cc)/dMw_j = (F_j B(alpha) - B(alpha mu_F) + 2 Mw_j B(beta)
//                                - 2 B(beta mu_M)) / w^3,
//             times the trilinear derivative of M at x + u(x) (warp backward);
//             the result is g = N dL/du with L = -mean cc.
//   smooth    Gaussian of the raw gradient (Eulerian descent, Sec. 2.1).
//
// Framework: a block owns a 32 x TY column of outputs and marches along z
// through a chunk of cz planes.  For each input plane it stages a
// (TY+2R) x (32+2R) halo tile of the raw FP32 inputs in LDS (the next plane is
// already in flight in registers while the current one is reduced), reduces
// along y (expanding the raw inputs into the accumulated channels: for the
// forward pass the exact products F^2, Mw^2, F Mw in FP64) and then along x,
// and keeps the last 2R+1 plane sums in a register ring.  Box sums run a
// running sum through the ring; weighted stencils sum it with their taps.
#include "lmr_internal.h"

namespace lmr {

namespace {

constexpr int kTX = 32;
// element index whose byte offset lies beyond any channel (< 2^30 voxels)
constexpr unsigned kFarIndex = 0x3FFFFFFFu;

struct Tiling {
  int ty, tiles_x, tiles_y, nchunks, cz;
  int blocks() const { return tiles_x * tiles_y * nchunks; }
};

// z-chunk: long enough that the 2R halo planes of a chunk stay a small
// fraction when the volume is large, short enough that small volumes still
// give the launch a few hundred blocks.
Tiling make_tiling(const Geom& g, int ty) {
  Tiling t;
  t.ty = ty;
  t.tiles_x = (g.nx + kTX - 1) / kTX;
  t.tiles_y = (g.ny + ty - 1) / ty;
  const int tiles = t.tiles_x * t.tiles_y;
  const int want = (2048 + tiles - 1) / tiles;
  int cz = (g.nz + want - 1) / want;
  if (tiles * ((g.nz + 15) / 16) >= 1024 && cz < 16) cz = 16;
  if (cz < 4) cz = 4;
  if (cz > g.nz) cz = g.nz;
  t.cz = cz;
  t.nchunks = (g.nz + cz - 1) / cz;
  return t;
}

template <int R, int TY, class P>
__global__ void __launch_bounds__(kTX* TY)
    k_stencil(const P pol, Geom g, int cz, int tiles_x, int tiles_y) {
  using A = typename P::Acc;
  constexpr int NR = P::NRAW, NC = P::NCH;
  constexpr int W = 2 * R + 1, LX = kTX + 2 * R, LY = TY + 2 * R, NT = kTX * TY;
  constexpr int NPOS = LX * LY, PER = (NPOS + NT - 1) / NT;
  __shared__ float s_in[NR][LY][LX];
  __shared__ A s_y[NC][TY][LX];

  if (!pol.active()) return;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tx_i = b % tiles_x;
  const int ty_i = (b / tiles_x) % tiles_y;
  const int ch = b / (tiles_x * tiles_y);
  const int x0 = tx_i * kTX, y0 = ty_i * TY, z0 = ch * cz;
  const int z1 = min(z0 + cz, g.nz);
  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool own = gx < g.nx && gy < g.ny;
  const int plane = g.ny * g.nx;

  // positions of the halo tile this thread stages, and their raw values
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
  typename P::Local loc = pol.begin_block();
  // Branch-free staging: a padding position reads kFarIndex and a plane
  // outside the volume wraps beyond the buffer; both read 0.
  float pre[PER][NR];
  auto fetch = [&](int zi) {
    const unsigned zoff = static_cast<unsigned>(zi * plane);
#pragma unroll
    for (int p = 0; p < PER; ++p)
      pol.load(loc, pin[p] ? zoff + static_cast<unsigned>(pidx[p]) : kFarIndex, pre[p]);
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
    run[c] = A(0);
#pragma unroll
    for (int k = 0; k < W; ++k) ring[k][c] = A(0);
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
          for (int c = 0; c < NC; ++c) a[c] = A(0);
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
        for (int c = 0; c < NC; ++c) pl[c] = A(0);
#pragma unroll
        for (int k = 0; k < W; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) pl[c] += pol.wt(k) * s_y[c][ly][lx + k];
        A sm[NC];
        if (P::kBox) {
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
            for (int c = 0; c < NC; ++c) sm[c] += pol.wt(k) * ring[(s + 1 + k) % W][c];
        }
        const int zo = zi - R;
        if (zo >= z0 && own) pol.emit(loc, zo * plane + gy * g.nx + gx, gx, gy, zo, sm);
      }
      ++zi;
    }
  }
  pol.end_block(loc);
}

// Block sum of one double per thread, written to out[blockIdx.x].
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
    out[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------- forward (P2)
template <typename T, int NT>
struct FwdPol {
  using Acc = double;
  static constexpr int NRAW = 2, NCH = 5;
  static constexpr bool kBox = true;
  const T* __restrict__ F;
  const float* __restrict__ Mw;
  float* __restrict__ maps;
  float* __restrict__ cc;
  double* __restrict__ partials;
  const DevState* st;
  int N;
  double inv_n, eps;
  struct Local {
    double sum;
    RBuf bF, bM;
  };

  __device__ bool active() const { return !st || !st->stalled; }
  __device__ static constexpr double wt(int) { return 1.0; }
  __device__ Local begin_block() const {
    return Local{0.0, make_rbuf_n(F, N), make_rbuf_n(Mw, N)};
  }
  __device__ void load(const Local& l, unsigned i, float v[2]) const {
    v[0] = bld<T>(l.bF, i);
    v[1] = bld<float>(l.bM, i);
  }
  __device__ void accum(double a[5], const float r[2], int) const {
    const double f = r[0], m = r[1];
    a[0] += f;
    a[1] += m;
    a[2] = fma(f, f, a[2]);
    a[3] = fma(m, m, a[3]);
    a[4] = fma(f, m, a[4]);
  }
  __device__ void emit(Local& loc, int i, int, int, int, const double S[5]) const {
    const double muF = S[0] * inv_n, muM = S[1] * inv_n;
    const double sfm = S[4] * inv_n - muF * muM;
    const double sff = S[2] * inv_n - muF * muF;
    const double smm = S[3] * inv_n - muM * muM;
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
  __device__ void end_block(const Local& loc) const { block_sum_to<NT>(loc.sum, partials); }
};

// ------------------------------------------------------------ backward (P4)
template <typename T>
struct BwdPol {
  using Acc = double;
  static constexpr int NRAW = 4, NCH = 4;
  static constexpr bool kBox = true;
  const T* __restrict__ F;
  const T* __restrict__ M;
  const float* __restrict__ Mw;
  const float* __restrict__ maps;
  const float* U0;
  const float* U1;
  const float* u_explicit;
  float* __restrict__ graw;
  const DevState* st;
  Geom g;
  double inv_n;
  struct Local {
    const float* u;
    RBuf bmap[4];
    RBuf bM;
  };

  __device__ bool active() const { return !st || (!st->stalled && st->accepted); }
  __device__ static constexpr double wt(int) { return 1.0; }
  __device__ Local begin_block() const {
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
  __device__ void accum(double a[4], const float r[4], int) const {
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] += static_cast<double>(r[c]);
  }
  __device__ void emit(const Local& loc, int i, int x, int y, int z,
                       const double B[4]) const {
    const int N = static_cast<int>(g.N);
    const float* u = loc.u;
    const double fj = ldf(F, i), mj = Mw[i];
    const double dS = (fj * B[0] - B[1] + 2.0 * mj * B[2] - 2.0 * B[3]) * inv_n;
    const float d = static_cast<float>(dS);
    float gm[3], v[8];
    const BCell c = make_bcell(g, x, y, z, u[i], u[N + i], u[2 * N + i]);
    bcorners<T>(loc.bM, g, c, v);
    binterp(c, v, gm);
    graw[i] = -d * gm[0];
    graw[N + i] = -d * gm[1];
    graw[2 * N + i] = -d * gm[2];
  }
  __device__ void end_block(const Local&) const {}
};

// ----------------------------------------------------------- smoothing (P5)
template <int R>
struct SmoothPol {
  using Acc = float;
  static constexpr int NRAW = 3, NCH = 3;
  static constexpr bool kBox = false;
  const float* __restrict__ in;
  float* __restrict__ out;
  const DevState* st;
  int N;
  float w[2 * R + 1];
  struct Local {
    RBuf b[3];
  };

  __device__ bool active() const { return !st || (!st->stalled && st->accepted); }
  __device__ float wt(int k) const { return w[k]; }
  __device__ Local begin_block() const {
    return Local{{make_rbuf_n(in, N), make_rbuf_n(in + N, N), make_rbuf_n(in + 2 * N, N)}};
  }
  __device__ void load(const Local& l, unsigned i, float v[3]) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = bld<float>(l.b[c], i);
  }
  __device__ void accum(float a[3], const float r[3], int k) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) a[c] += w[k] * r[c];
  }
  __device__ void emit(Local&, int i, int, int, int, const float S[3]) const {
    out[i] = S[0];
    out[N + i] = S[1];
    out[2 * N + i] = S[2];
  }
  __device__ void end_block(const Local&) const {}
};

constexpr int kTY = 8;

template <class P, int R>
hipError_t run(const P& pol, const Geom& g, hipStream_t s) {
  Tiling t = make_tiling(g, kTY);
  hipLaunchKernelGGL((k_stencil<R, kTY, P>), dim3(t.blocks()), dim3(kTX * kTY), 0, s,
                     pol, g, t.cz, t.tiles_x, t.tiles_y);
  return hipGetLastError();
}

template <class P>
hipError_t run_box(const P& pol, int window, const Geom& g, hipStream_t s) {
  switch (window / 2) {
    case 1: return run<P, 1>(pol, g, s);
    case 2: return run<P, 2>(pol, g, s);
    case 3: return run<P, 3>(pol, g, s);
    case 4: return run<P, 4>(pol, g, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t fwd_t(const T* F, const float* Mw, const Geom& g, const lmr_params& p,
                 const DevState* st, float* maps, double* partials, float* cc,
                 hipStream_t s) {
  FwdPol<T, kTX * kTY> pol;
  pol.F = F;
  pol.Mw = Mw;
  pol.maps = maps;
  pol.cc = cc;
  pol.partials = partials;
  pol.st = st;
  pol.N = static_cast<int>(g.N);
  pol.inv_n = 1.0 / ((double)p.window * p.window * p.window);
  pol.eps = p.cc_eps;
  return run_box(pol, p.window, g, s);
}

template <typename T>
hipError_t bwd_t(const T* F, const T* M, const float* Mw, const float* maps,
                 const Geom& g, const lmr_params& p, const DevState* st,
                 const float* U0, const float* U1, const float* ue, float* graw,
                 hipStream_t s) {
  BwdPol<T> pol;
  pol.F = F;
  pol.M = M;
  pol.Mw = Mw;
  pol.maps = maps;
  pol.U0 = U0;
  pol.U1 = U1;
  pol.u_explicit = ue;
  pol.graw = graw;
  pol.st = st;
  pol.g = g;
  pol.inv_n = 1.0 / ((double)p.window * p.window * p.window);
  return run_box(pol, p.window, g, s);
}

template <int R>
hipError_t smooth_r(const float* in, float* out, const Geom& g, double sigma,
                    const DevState* st, hipStream_t s) {
  SmoothPol<R> pol;
  pol.in = in;
  pol.out = out;
  pol.st = st;
  pol.N = static_cast<int>(g.N);
  double w[2 * R + 1], tot = 0.0;
  for (int k = -R; k <= R; ++k) {
    w[k + R] = R == 0 ? 1.0 : exp(-(double)k * k / (2.0 * sigma * sigma));
    tot += w[k + R];
  }
  for (int k = 0; k <= 2 * R; ++k) pol.w[k] = static_cast<float>(w[k] / tot);
  return run<SmoothPol<R>, R>(pol, g, s);
}

}  // namespace

int fwd_num_blocks(const Geom& g, int) { return make_tiling(g, kTY).blocks(); }

int gauss_radius(double sigma) {
  if (!(sigma > 0.0)) return 0;
  return (int)ceil(3.0 * sigma - 1e-12);
}

hipError_t launch_fwd(const void* F, lmr_dtype t, const float* Mw, const Geom& g,
                      const lmr_params& p, const DevState* st, float* maps,
                      double* partials, float* cc_map, hipStream_t s) {
  if (t == LMR_BF16)
    return fwd_t(static_cast<const uint16_t*>(F), Mw, g, p, st, maps, partials, cc_map,
                 s);
  return fwd_t(static_cast<const float*>(F), Mw, g, p, st, maps, partials, cc_map, s);
}

hipError_t launch_bwd(const void* F, const void* M, lmr_dtype t, const float* Mw,
                      const float* maps, const Geom& g, const lmr_params& p,
                      const DevState* st, const float* U0, const float* U1,
                      const float* ue, float* graw, hipStream_t s) {
  if (t == LMR_BF16)
    return bwd_t(static_cast<const uint16_t*>(F), static_cast<const uint16_t*>(M), Mw,
                 maps, g, p, st, U0, U1, ue, graw, s);
  return bwd_t(static_cast<const float*>(F), static_cast<const float*>(M), Mw, maps, g,
               p, st, U0, U1, ue, graw, s);
}

hipError_t launch_smooth(const float* graw, const Geom& g, const lmr_params& p,
                         const DevState* st, float* out, hipStream_t s) {
  switch (gauss_radius(p.grad_sigma)) {
    case 0: return smooth_r<0>(graw, out, g, p.grad_sigma, st, s);
    case 1: return smooth_r<1>(graw, out, g, p.grad_sigma, st, s);
    case 2: return smooth_r<2>(graw, out, g, p.grad_sigma, st, s);
    case 3: return smooth_r<3>(graw, out, g, p.grad_sigma, st, s);
    case 4: return smooth_r<4>(graw, out, g, p.grad_sigma, st, s);
    case 5: return smooth_r<5>(graw, out, g, p.grad_sigma, st, s);
    case 6: return smooth_r<6>(graw, out, g, p.grad_sigma, st, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lmr
