// Squared-error similarity of one LM attempt (Sec. 2.2: the mean squared
// error is already a squared loss) and the Demons variant of the step
// (Sec. 2.3, eq. demons).
//
//   k_mse_fwd      L = mean (F - Mw)^2: one FP64 partial of -sum (F - Mw)^2
//                  per block in a fixed order (the decision reduces them)
//   k_mse_bwd      g = N dr/du with the scalar residual r = sqrt(L):
//                  g_j = (Mw_j - F_j) dMw_j / r   (0 where r = 0)
//   k_demons_force du_x = r_x n_x / (|n_x|^2 + lambda) with the per-voxel
//                  residual r_x = F - Mw and n_x = grad M at x + u(x) of the
//                  accepted field (eq. demons, global lambda)
//   k_demons_keep  stores r_x and n_x of a newly accepted field
#include "lmr_internal.h"

namespace lmr {

namespace {

constexpr int kMseThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kMseThreads)
    k_mse_fwd(const T* __restrict__ F, const float* __restrict__ Mw, long long N,
              double* __restrict__ partials, float* __restrict__ sq_map,
              const DevState* __restrict__ st) {
  if (st && st->stalled) return;
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)kMseThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kMseThreads) {
    const double d = static_cast<double>(ldf(F, static_cast<int>(i))) - Mw[i];
    const double q = d * d;
    if (sq_map) sq_map[i] = static_cast<float>(q);
    s += q;
  }
  __shared__ double red[kMseThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kMseThreads / 64; ++k) t += red[k];
    partials[blockIdx.x] = -t;  // the decision forms L = -sum / N
  }
}

// need: 2 = only after an acceptance.  r: the state's residual, or sqrt of
// *loss (explicit mode).
template <typename T>
__global__ void __launch_bounds__(kMseThreads)
    k_mse_bwd(const T* __restrict__ F, const float* __restrict__ Mw, const float* dMw,
              long long N, const DevState* __restrict__ st, const double* __restrict__ loss,
              float* graw) {
  if (st) {
    if (st->stalled || !st->accepted) return;
  }
  const double r = st ? st->r : sqrt(fmax(*loss, 0.0));
  const float inv = r > 0.0 ? static_cast<float>(1.0 / r) : 0.0f;
  for (long long i = blockIdx.x * (long long)kMseThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kMseThreads) {
    const float d = (Mw[i] - ldf(F, static_cast<int>(i))) * inv;
    const float n0 = dMw[i], n1 = dMw[N + i], n2 = dMw[2 * N + i];
    graw[i] = d * n0;
    graw[N + i] = d * n1;
    graw[2 * N + i] = d * n2;
  }
}

__global__ void __launch_bounds__(kMseThreads)
    k_demons_force(const float* __restrict__ keep, long long N,
                   const DevState* __restrict__ st, float* __restrict__ du) {
  if (st->stalled) return;
  const float lam = static_cast<float>(st->lambda);
  for (long long i = blockIdx.x * (long long)kMseThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kMseThreads) {
    const float r = keep[i];
    const float n0 = keep[N + i], n1 = keep[2 * N + i], n2 = keep[3 * N + i];
    const float s = r / fmaf(n2, n2, fmaf(n1, n1, fmaf(n0, n0, lam)));
    du[i] = s * n0;
    du[N + i] = s * n1;
    du[2 * N + i] = s * n2;
  }
}

// keep = [r_x | n_x] ([4][N]) of the accepted field: need = 2 only after an
// acceptance (state mode), always without a state.
template <typename T>
__global__ void __launch_bounds__(kMseThreads)
    k_demons_keep(const T* __restrict__ F, const float* __restrict__ Mw,
                  const float* __restrict__ dMw, long long N, const DevState* __restrict__ st,
                  float* __restrict__ keep) {
  if (st && (st->stalled || !st->accepted)) return;
  for (long long i = blockIdx.x * (long long)kMseThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kMseThreads) {
    keep[i] = ldf(F, static_cast<int>(i)) - Mw[i];
    keep[N + i] = dMw[i];
    keep[2 * N + i] = dMw[N + i];
    keep[3 * N + i] = dMw[2 * N + i];
  }
}

unsigned blocks_for(long long N) {
  long long b = (N + kMseThreads - 1) / kMseThreads;
  if (b > 4096) b = 4096;
  return static_cast<unsigned>(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_mse_fwd(const void* F, lmr_dtype t, const float* Mw, const Geom& g,
                          int nparts, double* partials, float* sq_map, const DevState* st,
                          hipStream_t s) {
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_mse_fwd<uint16_t>, dim3(nparts), dim3(kMseThreads), 0, s,
                       static_cast<const uint16_t*>(F), Mw, g.N, partials, sq_map, st);
  else
    hipLaunchKernelGGL(k_mse_fwd<float>, dim3(nparts), dim3(kMseThreads), 0, s,
                       static_cast<const float*>(F), Mw, g.N, partials, sq_map, st);
  return hipGetLastError();
}

hipError_t launch_mse_bwd(const void* F, lmr_dtype t, const float* Mw, const float* dMw,
                          const Geom& g, const DevState* st, const double* loss, float* graw,
                          hipStream_t s) {
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_mse_bwd<uint16_t>, dim3(blocks_for(g.N)), dim3(kMseThreads), 0, s,
                       static_cast<const uint16_t*>(F), Mw, dMw, g.N, st, loss, graw);
  else
    hipLaunchKernelGGL(k_mse_bwd<float>, dim3(blocks_for(g.N)), dim3(kMseThreads), 0, s,
                       static_cast<const float*>(F), Mw, dMw, g.N, st, loss, graw);
  return hipGetLastError();
}

hipError_t launch_demons_force(const float* keep, const Geom& g, const DevState* st,
                               float* du, hipStream_t s) {
  hipLaunchKernelGGL(k_demons_force, dim3(blocks_for(g.N)), dim3(kMseThreads), 0, s, keep,
                     g.N, st, du);
  return hipGetLastError();
}

hipError_t launch_demons_keep(const void* F, lmr_dtype t, const float* Mw, const float* dMw,
                              const Geom& g, const DevState* st, float* keep,
                              hipStream_t s) {
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_demons_keep<uint16_t>, dim3(blocks_for(g.N)), dim3(kMseThreads), 0,
                       s, static_cast<const uint16_t*>(F), Mw, dMw, g.N, st, keep);
  else
    hipLaunchKernelGGL(k_demons_keep<float>, dim3(blocks_for(g.N)), dim3(kMseThreads), 0, s,
                       static_cast<const float*>(F), Mw, dMw, g.N, st, keep);
  return hipGetLastError();
}

}  // namespace lmr
