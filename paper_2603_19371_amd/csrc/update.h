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
template <typename T, int V>
__device__ __forceinline__ void update_voxels(const T* __restrict__ M, const Geom& g,
                                              const UpdateArgs& a, int x, int y, int z0) {
  const int N = static_cast<int>(g.N);
  int idx[V];
  bool ok[V];
  float e[V][3], n[V][3], mw[V], dm[V][3];
#pragma unroll
  for (int j = 0; j < V; ++j) {
    ok[j] = z0 + j < g.nz;
    idx[j] = ((ok[j] ? z0 + j : z0) * g.ny + y) * g.nx + x;
    const int i = idx[j];
    const float g0 = a.G[i], g1 = a.G[N + i], g2 = a.G[2 * N + i];
    const float s = -a.r / fmaf(g2, g2, fmaf(g1, g1, fmaf(g0, g0, a.lam)));
    e[j][0] = a.eps * (s * g0);
    e[j][1] = a.eps * (s * g1);
    e[j][2] = a.eps * (s * g2);
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
