// Per-voxel step of one LM attempt, shared by the per-pair update kernel and
// the batched persistent kernel:
//   du = -r g / (|g|^2 + lambda)                 (Sec. 2.2, eq. tile1)
//   u~ = eps du + u o (Id + eps du)              (Sec. 2.1, eq. compositive)
//   Mw = M o (Id + u~)                           (the candidate's warped image)
#pragma once

#include "lmr_internal.h"

namespace lmr {

struct UpdateArgs {
  const float* uin;  // accepted field [3][N]
  float* uo;         // candidate field [3][N]
  const float* G;    // smoothed gradient of the accepted field [3][N]
  float* Mw;         // warped moving image at the candidate (null: skip)
  float* dMw;        // its spatial derivative [3][N] (null: skip), for P4
  float r, lam, eps;
  int compositive;
};

// ----------------------------------------------------------- step policies
// The direction e = eps du of one voxel from the accepted state.  A policy
// loads its per-voxel operands (load: element index i, kFarIndex reads 0)
// ahead of their use and forms the direction (apply).
//   PointStep  du = -r g / (|g|^2 + lambda)                   (eq. tile1)
//   TileStep   du = -r (H_tile + lambda I)^-1 g               (eq. tilen)
//   AdamStep   du = -lr mhat / (sqrt(vhat) + eps_a), the moments of g
//              updated in place (the Adam comparator)
struct PointStep {
  const float* G;  // smoothed gradient of the accepted field [3][N]
  int N;
  float r, lam, eps;
  struct Regs {
    float g[3];
  };
  __device__ void load(unsigned i, Regs& q) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) q.g[c] = bld<float>(make_rbuf_n(G + c * N, N), i);
  }
  __device__ void apply(const Regs& q, int, int, int, int, float e[3]) const {
    const float g0 = q.g[0], g1 = q.g[1], g2 = q.g[2];
    const float s = -r / fmaf(g2, g2, fmaf(g1, g1, fmaf(g0, g0, lam)));
    e[0] = eps * (s * g0);
    e[1] = eps * (s * g1);
    e[2] = eps * (s * g2);
  }
};

// Pooled Hessian of the voxel's tile (side k, tiles from the origin, x
// fastest; H holds the mean of g g^T over the tile as xx, yy, zz, xy, xz, yz
// in FP64).  The symmetric 3x3 system is solved by its adjugate in FP64;
// H + lambda I is positive definite for lambda > 0.
struct TileStep {
  const float* G;
  const double* H;
  int N, k, tx, ty;
  double r, lam;
  float eps;
  using Regs = PointStep::Regs;
  __device__ void load(unsigned i, Regs& q) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) q.g[c] = bld<float>(make_rbuf_n(G + c * N, N), i);
  }
  __device__ void apply(const Regs& q, int, int x, int y, int z, float e[3]) const {
    const double* h = H + 6 * (((z / k) * ty + y / k) * tx + x / k);
    const double a = h[0] + lam, b = h[1] + lam, c = h[2] + lam;
    const double d = h[3], f = h[4], o = h[5];  // xy, xz, yz
    const double c00 = b * c - o * o, c01 = f * o - d * c, c02 = d * o - b * f;
    const double c11 = a * c - f * f, c12 = d * f - a * o, c22 = a * b - d * d;
    const double det = a * c00 + d * c01 + f * c02;
    const double s = -r / det;
    const double g0 = q.g[0], g1 = q.g[1], g2 = q.g[2];
    e[0] = eps * static_cast<float>(s * (c00 * g0 + c01 * g1 + c02 * g2));
    e[1] = eps * static_cast<float>(s * (c01 * g0 + c11 * g1 + c12 * g2));
    e[2] = eps * static_cast<float>(s * (c02 * g0 + c12 * g1 + c22 * g2));
  }
};

// Adam on the smoothed gradient: m <- b1 m + (1 - b1) g, v <- b2 v +
// (1 - b2) g^2, du = -lr (m / c1) / (sqrt(v / c2) + eps_a) with the bias
// corrections c1 = 1 - b1^t, c2 = 1 - b2^t of step t.
struct AdamStep {
  const float* G;
  float* m;  // first moments [3][N], updated in place
  float* v;  // second moments [3][N], updated in place
  int N;
  float b1, ob1, b2, ob2, c1, c2, lr, aeps, eps;  // ob = 1 - b
  struct Regs {
    float g[3], m[3], v[3];
  };
  __device__ void load(unsigned i, Regs& q) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q.g[c] = bld<float>(make_rbuf_n(G + c * N, N), i);
      q.m[c] = bld<float>(make_rbuf_n(m + c * N, N), i);
      q.v[c] = bld<float>(make_rbuf_n(v + c * N, N), i);
    }
  }
  __device__ void apply(const Regs& q, int i, int, int, int, float e[3]) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float mn = b1 * q.m[c] + ob1 * q.g[c];
      const float vn = b2 * q.v[c] + ob2 * (q.g[c] * q.g[c]);
      m[c * N + i] = mn;
      v[c * N + i] = vn;
      const float d = -lr * (mn / c1) / (sqrtf(vn / c2) + aeps);
      e[c] = eps * d;
    }
  }
};

// A given direction field V (the smoothed Demons step, eq. demons): e = eps V.
struct GivenStep {
  const float* V;
  int N;
  float eps;
  using Regs = PointStep::Regs;
  __device__ void load(unsigned i, Regs& q) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) q.g[c] = bld<float>(make_rbuf_n(V + c * N, N), i);
  }
  __device__ void apply(const Regs& q, int, int, int, int, float e[3]) const {
    e[0] = eps * q.g[0];
    e[1] = eps * q.g[1];
    e[2] = eps * q.g[2];
  }
};

template <typename T>
__device__ __forceinline__ void update_voxel(const T* __restrict__ M, const Geom& g,
                                             const UpdateArgs& a, int x, int y, int z) {
  const int N = static_cast<int>(g.N);
  const int i = (z * g.ny + y) * g.nx + x;
  const float g0 = a.G[i], g1 = a.G[N + i], g2 = a.G[2 * N + i];
  const float s = -a.r / fmaf(g2, g2, fmaf(g1, g1, fmaf(g0, g0, a.lam)));
  const float e0 = a.eps * (s * g0), e1 = a.eps * (s * g1), e2 = a.eps * (s * g2);
  float b0, b1, b2;
  if (a.compositive) {
    const BCell c = make_bcell(g, x, y, z, e0, e1, e2);
    float v[8];
    bcorners<float>(make_rbuf_n(a.uin, N), g, c, v);
    b0 = binterp(c, v, nullptr);
    bcorners<float>(make_rbuf_n(a.uin + N, N), g, c, v);
    b1 = binterp(c, v, nullptr);
    bcorners<float>(make_rbuf_n(a.uin + 2 * N, N), g, c, v);
    b2 = binterp(c, v, nullptr);
  } else {
    b0 = a.uin[i];
    b1 = a.uin[N + i];
    b2 = a.uin[2 * N + i];
  }
  const float n0 = e0 + b0, n1 = e1 + b1, n2 = e2 + b2;
  a.uo[i] = n0;
  a.uo[N + i] = n1;
  a.uo[2 * N + i] = n2;
  if (M && a.Mw) {
    const BCell c = make_bcell(g, x, y, z, n0, n1, n2);
    float v[8], d[3];
    bcorners<T>(make_rbuf_n(M, N), g, c, v);
    a.Mw[i] = binterp(c, v, a.dMw ? d : nullptr);
    if (a.dMw) {
      a.dMw[i] = d[0];
      a.dMw[N + i] = d[1];
      a.dMw[2 * N + i] = d[2];
    }
  }
}

// The same step for the voxels (x, y, z0 + j), j < V, z0 + j < nz, of one
// thread, in phases (all gradient loads, then all field gathers, then all
// image gathers, then the stores), so that the gathers of the V voxels are in
// flight together: the step is bound by the latency of its two dependent
// gathers, not by bandwidth.  Per voxel the arithmetic is that of
// update_voxel, bit for bit.
template <typename T, int V, class S>
__device__ __forceinline__ void update_voxels(const T* __restrict__ M, const Geom& g,
                                              const UpdateArgs& a, const S& step, int x,
                                              int y, int z0) {
  const int N = static_cast<int>(g.N);
  int idx[V];
  bool ok[V];
  float e[V][3], n[V][3], mw[V], dm[V][3];
  typename S::Regs q[V];
#pragma unroll
  for (int j = 0; j < V; ++j) {
    ok[j] = z0 + j < g.nz;
    idx[j] = ((ok[j] ? z0 + j : z0) * g.ny + y) * g.nx + x;
    step.load(static_cast<unsigned>(idx[j]), q[j]);
  }
#pragma unroll
  for (int j = 0; j < V; ++j) {
    e[j][0] = e[j][1] = e[j][2] = 0.0f;
    if (ok[j]) step.apply(q[j], idx[j], x, y, z0 + j, e[j]);
  }
  if (a.compositive) {
    const RBuf b0 = make_rbuf_n(a.uin, N), b1 = make_rbuf_n(a.uin + N, N),
               b2 = make_rbuf_n(a.uin + 2 * N, N);
    float v[V][3][8];
    BCell c[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      c[j] = make_bcell(g, x, y, ok[j] ? z0 + j : z0, e[j][0], e[j][1], e[j][2]);
      bcorners<float>(b0, g, c[j], v[j][0]);
      bcorners<float>(b1, g, c[j], v[j][1]);
      bcorners<float>(b2, g, c[j], v[j][2]);
    }
#pragma unroll
    for (int j = 0; j < V; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) n[j][k] = e[j][k] + binterp(c[j], v[j][k], nullptr);
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) n[j][k] = e[j][k] + a.uin[k * N + idx[j]];
  }
  if (M && a.Mw) {
    const RBuf bm = make_rbuf_n(M, N);
    float v[V][8];
    BCell c[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      c[j] = make_bcell(g, x, y, ok[j] ? z0 + j : z0, n[j][0], n[j][1], n[j][2]);
      bcorners<T>(bm, g, c[j], v[j]);
    }
#pragma unroll
    for (int j = 0; j < V; ++j) mw[j] = binterp(c[j], v[j], a.dMw ? dm[j] : nullptr);
  }
#pragma unroll
  for (int j = 0; j < V; ++j) {
    if (!ok[j]) continue;
    const int i = idx[j];
    a.uo[i] = n[j][0];
    a.uo[N + i] = n[j][1];
    a.uo[2 * N + i] = n[j][2];
    if (M && a.Mw) {
      a.Mw[i] = mw[j];
      if (a.dMw) {
        a.dMw[i] = dm[j][0];
        a.dMw[N + i] = dm[j][1];
        a.dMw[2 * N + i] = dm[j][2];
      }
    }
  }
}

// The attempt step with the accepted field staged in LDS.  A block owns
// a 32 x 8 column of voxels and marches along z through a chunk of planes,
// keeping the planes z-1, z, z+1 of the three field channels (with a
// one-voxel halo in x and y) in a ring of LDS slots.  The compositive
// gather u(x + eps du) reads its eight corners from LDS whenever every
// component of eps du lies in [-1, 1) (the cell's corners are then within one
// voxel of x), and from memory otherwise.  The staged values are the field's
// own, and out-of-volume corners carry weight 0 either way, so each voxel's
// result is that of update_voxel (up to the sign of an exact zero).
constexpr int kSX = 32, kSY = 8, kSNT = kSX * kSY;
constexpr int kSLX = kSX + 2, kSLY = kSY + 2, kSPOS = kSLX * kSLY;
constexpr int kSPER = (kSPOS + kSNT - 1) / kSNT;
constexpr int kSlots = 4;  // planes z-1..z+1 in use while z+2 is written


struct StagedLds {
  float u[kSlots][3][kSLY][kSLX];  // plane slot, channel, row, column
};

// One tile of the staged update: voxels [bx, bx+32) x [by, by+8) x [z0, z1)
// (clipped to the volume), with a block of 256 threads, in the LDS `sm`.
template <typename T, class S>
__device__ __forceinline__ void staged_update_tile(const T* __restrict__ M, const Geom& g,
                                                   const UpdateArgs& a, const S& step,
                                                   int bx, int by, int z0, int z1,
                                                   StagedLds& sm) {
  auto& s_u = sm.u;
  // a block that runs tiles back to back: every thread is done with the
  // previous tile's slots before they are overwritten
  __syncthreads();
  const int N = static_cast<int>(g.N), plane = g.nx * g.ny;
  const int lx = threadIdx.x % kSX, ly = threadIdx.x / kSX;
  const int x = bx + lx, y = by + ly;
  const bool own = x < g.nx && y < g.ny;
  const RBuf bu[3] = {make_rbuf_n(a.uin, N), make_rbuf_n(a.uin + N, N),
                      make_rbuf_n(a.uin + 2 * N, N)};

  // staged positions of this thread (padding positions read 0)
  int pidx[kSPER];
  bool pin[kSPER];
#pragma unroll
  for (int p = 0; p < kSPER; ++p) {
    const int i = threadIdx.x + p * kSNT;
    const int yy = i / kSLX, xx = i - yy * kSLX;
    const int gy = by - 1 + yy, gx = bx - 1 + xx;
    pin[p] = i < kSPOS && (unsigned)gy < (unsigned)g.ny && (unsigned)gx < (unsigned)g.nx;
    pidx[p] = pin[p] ? gy * g.nx + gx : 0;
  }
  float pre[kSPER][3];
  auto fetch = [&](int zi) {
    const bool zin = (unsigned)zi < (unsigned)g.nz;
#pragma unroll
    for (int p = 0; p < kSPER; ++p) {
      const unsigned o = (zin && pin[p]) ? static_cast<unsigned>(zi * plane + pidx[p])
                                         : kFarIndex;
#pragma unroll
      for (int c = 0; c < 3; ++c) pre[p][c] = bld<float>(bu[c], o);
    }
  };
  auto slot = [](int zi) { return (zi + kSlots) % kSlots; };  // zi >= -1
  auto commit = [&](int zi) {
    const int sl = slot(zi);
#pragma unroll
    for (int p = 0; p < kSPER; ++p) {
      const int i = threadIdx.x + p * kSNT;
      if (i < kSPOS) {
        const int yy = i / kSLX, xx = i - yy * kSLX;
#pragma unroll
        for (int c = 0; c < 3; ++c) s_u[sl][c][yy][xx] = pre[p][c];
      }
    }
  };

  fetch(z0 - 1);
  commit(z0 - 1);
  fetch(z0);
  commit(z0);
  fetch(z0 + 1);
  const RBuf bm = make_rbuf_n(M, N);
  // the step operands of the next plane are in flight while a plane is
  // processed
  const unsigned col = own ? static_cast<unsigned>(y * g.nx + x) : kFarIndex;
  typename S::Regs qn;
  step.load(own ? static_cast<unsigned>(z0 * plane) + col : kFarIndex, qn);
  // The image gather M(x + u~) of a plane stays in flight while the next
  // plane's field work runs; it is finished (interpolated and stored) then.
  const bool warp = M && a.Mw;
  BCell pc;
  float pv[8];
  int pi = -1;  // voxel of the pending image gather (-1: none)
  auto finish = [&]() {
    if (pi < 0) return;
    float d[3];
    a.Mw[pi] = binterp(pc, pv, a.dMw ? d : nullptr);
    if (a.dMw) {
      a.dMw[pi] = d[0];
      a.dMw[N + pi] = d[1];
      a.dMw[2 * N + pi] = d[2];
    }
  };
  for (int z = z0; z < z1; ++z) {
    // slot(z+1) last held plane z-3, whose readers finished before the
    // barrier of the previous iteration
    commit(z + 1);
    if (z + 2 <= z1) fetch(z + 2);
    const typename S::Regs q = qn;
    if (z + 1 < z1)
      step.load(own ? static_cast<unsigned>((z + 1) * plane) + col : kFarIndex, qn);
    __syncthreads();
    if (!own) continue;
    const int i = (z * g.ny + y) * g.nx + x;
    float e[3];
    step.apply(q, i, x, y, z, e);
    const float e0 = e[0], e1 = e[1], e2 = e[2];
    const BCell c = make_bcell(g, x, y, z, e0, e1, e2);
    float b[3];
    if (e0 >= -1.0f && e0 < 1.0f && e1 >= -1.0f && e1 < 1.0f && e2 >= -1.0f && e2 < 1.0f) {
      // lower corner (x + floor(e0), y + floor(e1), z + floor(e2)), each
      // floor in {-1, 0}: staged column lx + floor + 1, row ly + floor + 1
      const int cx = lx + 1 + (e0 < 0.0f ? -1 : 0);
      const int cy = ly + 1 + (e1 < 0.0f ? -1 : 0);
      const int cz0 = z + (e2 < 0.0f ? -1 : 0);
      const int s0 = slot(cz0), s1 = slot(cz0 + 1);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float v[8];
        v[0] = s_u[s0][ch][cy][cx];
        v[1] = s_u[s0][ch][cy][cx + 1];
        v[2] = s_u[s0][ch][cy + 1][cx];
        v[3] = s_u[s0][ch][cy + 1][cx + 1];
        v[4] = s_u[s1][ch][cy][cx];
        v[5] = s_u[s1][ch][cy][cx + 1];
        v[6] = s_u[s1][ch][cy + 1][cx];
        v[7] = s_u[s1][ch][cy + 1][cx + 1];
        b[ch] = binterp(c, v, nullptr);
      }
    } else {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float v[8];
        bcorners<float>(bu[ch], g, c, v);
        b[ch] = binterp(c, v, nullptr);
      }
    }
    const float n0 = e0 + b[0], n1 = e1 + b[1], n2 = e2 + b[2];
    a.uo[i] = n0;
    a.uo[N + i] = n1;
    a.uo[2 * N + i] = n2;
    finish();
    if (warp) {
      pc = make_bcell(g, x, y, z, n0, n1, n2);
      bcorners<T>(bm, g, pc, pv);
      pi = i;
    }
  }
  if (own) finish();
}

template <typename T, class S>
__device__ __forceinline__ void staged_update_tile(const T* __restrict__ M, const Geom& g,
                                                   const UpdateArgs& a, const S& step,
                                                   int bx, int by, int z0, int z1) {
  __shared__ StagedLds sm;
  staged_update_tile(M, g, a, step, bx, by, z0, z1, sm);
}

// The rank-1 step of the update arguments (eq. tile1).
__device__ __forceinline__ PointStep point_step(const UpdateArgs& a, const Geom& g) {
  return PointStep{a.G, static_cast<int>(g.N), a.r, a.lam, a.eps};
}

// The update arguments of an attempt in state mode: the accepted field is
// U[cur], the candidate goes to the other buffer, r and lambda come from the
// device state.
__device__ __forceinline__ UpdateArgs update_args_from_state(const DevState* st,
                                                             float* U0, float* U1,
                                                             const float* G, float* Mw,
                                                             float eps, int compositive) {
  UpdateArgs a;
  const int cur = st->cur;
  a.uin = cur ? U1 : U0;
  a.uo = cur ? U0 : U1;
  a.G = G;
  a.Mw = Mw;
  a.dMw = nullptr;
  a.r = static_cast<float>(st->r);
  a.lam = static_cast<float>(st->lambda);
  a.eps = eps;
  a.compositive = compositive;
  return a;
}

}  // namespace lmr
