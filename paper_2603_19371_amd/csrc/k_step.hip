// Per-voxel kernels of one LM attempt and the on-device decision.
//
//   k_warp    Mw(x) = M(x + u(x))                       (Sec. 1, eq. 1)
//   k_update  du = -r g/(|g|^2 + lambda)                (Sec. 2.2, eq. tile1)
//             u~ = eps du + u o (Id + eps du)           (Sec. 2.1, eq. compositive)
//             Mw = M o (Id + u~)  (the candidate's warped image, fused here)
//   k_decide  FP64 loss reduction, damping rule and rejection test
//             (Sec. 2.2, eq. lambda-update / eq. delta-loss; Sec. 3.4, eq. rejection)
#include "lmr_internal.h"

#include <math.h>

namespace lmr {

namespace {

constexpr int kBX = 64, kBY = 4;

__device__ __forceinline__ bool voxel(const Geom& g, int& x, int& y, int& z, int& i) {
  x = blockIdx.x * kBX + threadIdx.x;
  y = blockIdx.y * kBY + threadIdx.y;
  z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return false;
  i = (z * g.ny + y) * g.nx + x;
  return true;
}

template <typename T>
__global__ void __launch_bounds__(kBX* kBY)
    k_warp(const T* __restrict__ M, const float* __restrict__ u, Geom g,
           float* __restrict__ Mw, float* __restrict__ dMw) {
  int x, y, z, i;
  if (!voxel(g, x, y, z, i)) return;
  const int N = static_cast<int>(g.N);
  const RBuf bm = make_rbuf_n(M, N);
  const BCell c = make_bcell(g, x, y, z, u[i], u[N + i], u[2 * N + i]);
  float v[8], d[3];
  bcorners<T>(bm, g, c, v);
  Mw[i] = binterp(c, v, dMw ? d : nullptr);
  if (dMw) {
    dMw[i] = d[0];
    dMw[N + i] = d[1];
    dMw[2 * N + i] = d[2];
  }
}

template <typename T>
__global__ void __launch_bounds__(kBX* kBY)
    k_update(const T* __restrict__ M, Geom g, const DevState* __restrict__ st,
             const float* __restrict__ G, float* U0, float* U1,
             const float* u_in, float* u_out, float r_arg, float lam_arg,
             float eps, int compositive, float* __restrict__ Mw) {
  const float* uin;
  float* uo;
  float r, lam;
  if (st) {
    if (st->stalled) return;
    const int cur = st->cur;
    uin = cur ? U1 : U0;
    uo = cur ? U0 : U1;
    r = static_cast<float>(st->r);
    lam = static_cast<float>(st->lambda);
  } else {
    uin = u_in;
    uo = u_out;
    r = r_arg;
    lam = lam_arg;
  }
  int x, y, z, i;
  if (!voxel(g, x, y, z, i)) return;
  const int N = static_cast<int>(g.N);
  const float g0 = G[i], g1 = G[N + i], g2 = G[2 * N + i];
  const float s = -r / (g0 * g0 + g1 * g1 + g2 * g2 + lam);
  const float e0 = eps * (s * g0), e1 = eps * (s * g1), e2 = eps * (s * g2);
  float b0, b1, b2;
  if (compositive) {
    const BCell c = make_bcell(g, x, y, z, e0, e1, e2);
    float v[8];
    bcorners<float>(make_rbuf_n(uin, N), g, c, v);
    b0 = binterp(c, v, nullptr);
    bcorners<float>(make_rbuf_n(uin + N, N), g, c, v);
    b1 = binterp(c, v, nullptr);
    bcorners<float>(make_rbuf_n(uin + 2 * N, N), g, c, v);
    b2 = binterp(c, v, nullptr);
  } else {
    b0 = uin[i];
    b1 = uin[N + i];
    b2 = uin[2 * N + i];
  }
  const float n0 = e0 + b0, n1 = e1 + b1, n2 = e2 + b2;
  uo[i] = n0;
  uo[N + i] = n1;
  uo[2 * N + i] = n2;
  if (M) {
    const BCell c = make_bcell(g, x, y, z, n0, n1, n2);
    float v[8];
    bcorners<T>(make_rbuf_n(M, N), g, c, v);
    Mw[i] = binterp(c, v, nullptr);
  }
}

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

constexpr int kDecideThreads = 256;

__global__ void __launch_bounds__(kDecideThreads)
    k_decide(DevState* st, const double* __restrict__ partials, int nparts,
             long long N, DecideParams dp, int mode, int force, double lambda0,
             double* probe) {
  if (mode == 0 && st->stalled) {
    if (threadIdx.x == 0) {
      st->accepted = 0;
    }
    return;
  }
  __shared__ double sh[kDecideThreads];
  double s = 0.0;
  for (int k = threadIdx.x; k < nparts; k += kDecideThreads) s += partials[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kDecideThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double L = -sh[0] / static_cast<double>(N);
  if (mode == 2) {
    *probe = L;
    return;
  }
  if (mode == 1) {
    st->lambda = lambda0;
    st->loss = L;
    st->loss_prev = L;
    st->cand_loss = L;
    st->r = 1.0 + L;
    st->n_hist = 1;
    st->retries = 0;
    st->accepted = 1;
    st->stalled = 0;
    st->cur = 0;
    st->attempts = 0;
    return;
  }
  st->cand_loss = L;
  st->attempts += 1;
  int acc;
  if (force >= 0) {
    acc = force ? 1 : 0;
  } else if (!isfinite(L)) {
    acc = 0;
  } else if (dp.tau < 0.0) {
    acc = 1;
  } else {
    double ref = st->n_hist >= 2 ? fabs(st->loss - st->loss_prev) : 0.0;
    acc = !((L - st->loss) > dp.tau * ref);
  }
  if (acc) {
    double f = (L > st->loss) ? dp.lambda_inc : dp.lambda_dec;
    st->lambda = clampd(f * st->lambda, dp.lambda_min, dp.lambda_max);
    st->loss_prev = st->loss;
    st->loss = L;
    st->r = 1.0 + L;
    st->n_hist += 1;
    st->retries = 0;
    st->cur = 1 - st->cur;
  } else {
    st->lambda = clampd(dp.lambda_inc * st->lambda, dp.lambda_min, dp.lambda_max);
    st->retries += 1;
    if (st->retries >= dp.max_retries && st->lambda >= dp.lambda_max) st->stalled = 1;
  }
  st->accepted = acc;
}

__global__ void k_copy_cur(const DevState* __restrict__ st, const float* U0,
                           const float* U1, float* __restrict__ dst, long long n) {
  const float* src = st->cur ? U1 : U0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_fill(float* __restrict__ dst, long long n, float v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = v;
}

dim3 vox_grid(const Geom& g) {
  return dim3((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY, g.nz);
}

}  // namespace

hipError_t launch_warp(const void* M, lmr_dtype t, const float* u, const Geom& g,
                       float* Mw, float* dMw, hipStream_t s) {
  dim3 blk(kBX, kBY);
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_warp<uint16_t>, vox_grid(g), blk, 0, s,
                       static_cast<const uint16_t*>(M), u, g, Mw, dMw);
  else
    hipLaunchKernelGGL(k_warp<float>, vox_grid(g), blk, 0, s,
                       static_cast<const float*>(M), u, g, Mw, dMw);
  return hipGetLastError();
}

hipError_t launch_update(const void* M, lmr_dtype t, const Geom& g,
                         const lmr_params& p, const DevState* st, const float* G,
                         float* U0, float* U1, const float* u_in, float* u_out,
                         double r, double lambda, float* Mw, hipStream_t s) {
  dim3 blk(kBX, kBY);
  float rf = static_cast<float>(r), lf = static_cast<float>(lambda);
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_update<uint16_t>, vox_grid(g), blk, 0, s,
                       static_cast<const uint16_t*>(M), g, st, G, U0, U1, u_in,
                       u_out, rf, lf, (float)p.step_eps, p.compositive, Mw);
  else
    hipLaunchKernelGGL(k_update<float>, vox_grid(g), blk, 0, s,
                       static_cast<const float*>(M), g, st, G, U0, U1, u_in, u_out,
                       rf, lf, (float)p.step_eps, p.compositive, Mw);
  return hipGetLastError();
}

hipError_t launch_decide(DevState* st, const double* partials, int nparts,
                         long long N, const DecideParams& dp, int mode, int force,
                         double lambda0, double* probe, hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(kDecideThreads), 0, s, st, partials,
                     nparts, N, dp, mode, force, lambda0, probe);
  return hipGetLastError();
}

hipError_t launch_copy_cur(const DevState* st, const float* U0, const float* U1,
                           float* dst, long long n, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_copy_cur, dim3((unsigned)blocks), dim3(256), 0, s, st, U0,
                     U1, dst, n);
  return hipGetLastError();
}

namespace {
__global__ void k_set_state(DevState* st, DevState v) {
  v.cur = st->cur;
  *st = v;
}
}  // namespace

hipError_t launch_set_state(DevState* st, const DevState& v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, s, st, v);
  return hipGetLastError();
}

hipError_t launch_fill(float* dst, long long n, float v, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, dst, n, v);
  return hipGetLastError();
}

}  // namespace lmr
