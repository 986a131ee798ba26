// Separable 3D stencils of one LM attempt, on a shared 2.5D framework.
//
//   k_fwd     LNCC forward: box sums of F, Mw, F^2, Mw^2, F Mw over the w^3
//             window (zero padding, divisor w^3), cc = s_FM^2/(s_FF s_MM + eps),
//             adjoint maps alpha = 2 s_FM/D, alpha mu_F, beta = -s_FM^2 s_FF/D^2,
//             beta mu_M, and one FP64 partial sum of cc per block.
//   k_bwd     LNCC backward: box sums of the four maps give
//             d(sum cc)/dMw_j = (F_j B(alpha) - B(alpha mu_F) + 2 Mw_j B(beta)
//                                - 2 B(beta mu_M)) / w^3,
//             times the trilinear derivative of M at x + u(x) (warp backward);
//             the result is g = N dL/du with L = -mean cc.
//   k_smooth  Gaussian of the raw gradient (Eulerian descent, Sec. 2.1).
//
// Framework: a block owns a TX x TY column of outputs and marches along z
// through a chunk of cz planes.  For each input plane it stages a
// (TY+2R) x (TX+2R) halo tile of the input channels in LDS, reduces along y
// then along x in LDS, and keeps the last 2R+1 plane sums in registers, whose
// weighted sum is the output plane R steps behind.  Box sums accumulate exact
// FP32 products in FP64.
#include "lmr_internal.h"

namespace lmr {

namespace {

constexpr int kTX = 32, kTY = 8;

struct Tiling {
  int tiles_x, tiles_y, nchunks, cz;
  int blocks() const { return tiles_x * tiles_y * nchunks; }
};

// Choose the z-chunk so that the launch has enough blocks to fill 256 CUs
// several times over while the z halo (2R extra planes per chunk) stays small.
Tiling make_tiling(const Geom& g) {
  Tiling t;
  t.tiles_x = (g.nx + kTX - 1) / kTX;
  t.tiles_y = (g.ny + kTY - 1) / kTY;
  int tiles = t.tiles_x * t.tiles_y;
  int want = (2048 + tiles - 1) / tiles;
  int cz = (g.nz + want - 1) / want;
  if (cz < 16) cz = 16;
  if (cz > g.nz) cz = g.nz;
  t.cz = cz;
  t.nchunks = (g.nz + cz - 1) / cz;
  return t;
}

template <int R, class P>
__global__ void __launch_bounds__(kTX* kTY)
    k_stencil(const P pol, Geom g, int cz, int tiles_x, int tiles_y) {
  using A = typename P::Acc;
  constexpr int NC = P::NCH;
  constexpr int W = 2 * R + 1, LX = kTX + 2 * R, LY = kTY + 2 * R, NT = kTX * kTY;
  __shared__ A s_in[NC][LY][LX];
  __shared__ A s_y[NC][kTY][LX];

  if (!pol.active()) return;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tx_i = b % tiles_x;
  const int ty_i = (b / tiles_x) % tiles_y;
  const int ch = b / (tiles_x * tiles_y);
  const int x0 = tx_i * kTX, y0 = ty_i * kTY, z0 = ch * cz;
  const int z1 = min(z0 + cz, g.nz);
  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool own = gx < g.nx && gy < g.ny;

  A ring[W][NC];
#pragma unroll
  for (int k = 0; k < W; ++k)
#pragma unroll
    for (int c = 0; c < NC; ++c) ring[k][c] = A(0);
  typename P::Local loc = pol.begin_block();

  for (int zi = z0 - R; zi < z1 + R; ++zi) {
    const bool zin = zi >= 0 && zi < g.nz;
    for (int i = threadIdx.x; i < LY * LX; i += NT) {
      const int yy = i / LX, xx = i - yy * LX;
      const int gyy = y0 - R + yy, gxx = x0 - R + xx;
      A v[NC];
      if (zin && (unsigned)gyy < (unsigned)g.ny && (unsigned)gxx < (unsigned)g.nx) {
        pol.load(((long long)zi * g.ny + gyy) * g.nx + gxx, v);
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = A(0);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) s_in[c][yy][xx] = v[c];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTY * LX; i += NT) {
      const int yy = i / LX, xx = i - yy * LX;
      A a[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) a[c] = A(0);
#pragma unroll
      for (int k = 0; k < W; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) a[c] += pol.wt(k) * s_in[c][yy + k][xx];
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
#pragma unroll
    for (int k = 0; k < W - 1; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) ring[k][c] = ring[k + 1][c];
#pragma unroll
    for (int c = 0; c < NC; ++c) ring[W - 1][c] = pl[c];
    const int zo = zi - R;
    if (zo >= z0 && own) {
      A sm[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) sm[c] = A(0);
#pragma unroll
      for (int k = 0; k < W; ++k)
#pragma unroll
        for (int c = 0; c < NC; ++c) sm[c] += pol.wt(k) * ring[k][c];
      pol.emit(loc, ((long long)zo * g.ny + gy) * g.nx + gx, gx, gy, zo, sm);
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
template <typename T>
struct FwdPol {
  using Acc = double;
  static constexpr int NCH = 5;
  const T* __restrict__ F;
  const float* __restrict__ Mw;
  float* __restrict__ maps;
  float* __restrict__ cc;
  double* __restrict__ partials;
  const DevState* st;
  long long N;
  double inv_n, eps;
  struct Local {
    double sum;
  };

  __device__ bool active() const { return !st || !st->stalled; }
  __device__ static constexpr double wt(int) { return 1.0; }
  __device__ Local begin_block() const { return Local{0.0}; }
  __device__ void load(long long i, double v[5]) const {
    const double f = ldf(F, i), m = Mw[i];
    v[0] = f;
    v[1] = m;
    v[2] = f * f;
    v[3] = m * m;
    v[4] = f * m;
  }
  __device__ void emit(Local& loc, long long i, int, int, int, const double S[5]) const {
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
  __device__ void end_block(const Local& loc) const {
    block_sum_to<kTX * kTY>(loc.sum, partials);
  }
};

// ------------------------------------------------------------ backward (P4)
template <typename T>
struct BwdPol {
  using Acc = double;
  static constexpr int NCH = 4;
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
  };

  __device__ bool active() const { return !st || (!st->stalled && st->accepted); }
  __device__ static constexpr double wt(int) { return 1.0; }
  __device__ Local begin_block() const {
    return Local{st ? (st->cur ? U1 : U0) : u_explicit};
  }
  __device__ void load(long long i, double v[4]) const {
    v[0] = maps[i];
    v[1] = maps[g.N + i];
    v[2] = maps[2 * g.N + i];
    v[3] = maps[3 * g.N + i];
  }
  __device__ void emit(const Local& loc, long long i, int x, int y, int z,
                       const double B[4]) const {
    const float* u = loc.u;
    const double fj = ldf(F, i), mj = Mw[i];
    const double dS = (fj * B[0] - B[1] + 2.0 * mj * B[2] - 2.0 * B[3]) * inv_n;
    const float d = static_cast<float>(dS);
    float gm[3];
    trilinear(M, g, x, y, z, u[i], u[g.N + i], u[2 * g.N + i], gm);
    graw[i] = -d * gm[0];
    graw[g.N + i] = -d * gm[1];
    graw[2 * g.N + i] = -d * gm[2];
  }
  __device__ void end_block(const Local&) const {}
};

// ----------------------------------------------------------- smoothing (P5)
template <int R>
struct SmoothPol {
  using Acc = float;
  static constexpr int NCH = 3;
  const float* __restrict__ in;
  float* __restrict__ out;
  const DevState* st;
  long long N;
  float w[2 * R + 1];
  struct Local {};

  __device__ bool active() const { return !st || (!st->stalled && st->accepted); }
  __device__ float wt(int k) const { return w[k]; }
  __device__ Local begin_block() const { return Local{}; }
  __device__ void load(long long i, float v[3]) const {
    v[0] = in[i];
    v[1] = in[N + i];
    v[2] = in[2 * N + i];
  }
  __device__ void emit(Local&, long long i, int, int, int, const float S[3]) const {
    out[i] = S[0];
    out[N + i] = S[1];
    out[2 * N + i] = S[2];
  }
  __device__ void end_block(const Local&) const {}
};

template <class P, int R>
hipError_t run(const P& pol, const Geom& g, hipStream_t s) {
  Tiling t = make_tiling(g);
  hipLaunchKernelGGL((k_stencil<R, P>), dim3(t.blocks()), dim3(kTX * kTY), 0, s, pol,
                     g, t.cz, t.tiles_x, t.tiles_y);
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
  FwdPol<T> pol;
  pol.F = F;
  pol.Mw = Mw;
  pol.maps = maps;
  pol.cc = cc;
  pol.partials = partials;
  pol.st = st;
  pol.N = g.N;
  const double n = (double)p.window * p.window * p.window;
  pol.inv_n = 1.0 / n;
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
  pol.N = g.N;
  double w[2 * R + 1], tot = 0.0;
  for (int k = -R; k <= R; ++k) {
    w[k + R] = R == 0 ? 1.0 : exp(-(double)k * k / (2.0 * sigma * sigma));
    tot += w[k + R];
  }
  for (int k = 0; k <= 2 * R; ++k) pol.w[k] = static_cast<float>(w[k] / tot);
  return run<SmoothPol<R>, R>(pol, g, s);
}

}  // namespace

int fwd_num_blocks(const Geom& g, int) { return make_tiling(g).blocks(); }

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
