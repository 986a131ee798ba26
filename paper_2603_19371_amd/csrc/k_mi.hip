// Mutual-information similarity of one LM attempt (Sec. 2.2: minimise
// (log2 B - MI)^2), from a B x B joint histogram with cubic B-spline Parzen
// windows.  Each image's values are mapped to bin coordinates
// 1 + (B - 3)(v - lo)/(hi - lo) ([lo, hi] its range over the volume, the
// moving range extended to 0, the value outside the volume), so every
// window's four bins lie inside [0, B).
//
//   k_mi_range   per-block minima and maxima of F and M; k_mi_range_final
//                turns them into the two affine maps (order-free: min/max)
//   k_mi_hist    per-block joint histograms of the window products (FP64),
//                summed
//                exactly as fixed-point integers (2^-32 per unit), so the
//                result does not depend on the order of the additions
//   k_mi_reduce  one block: the exact block sums, p, the marginals, MI (FP64,
//                fixed order) and the table log2(p_ab / p_b) of the gradient;
//                the decision reads N MI as its one partial (L = -MI)
//   k_mi_bwd     g = N dr/du = -(sum_ab w_a(F) w'_b(Mw) s_M log2(p_ab/p_b)) dMw
#include <algorithm>

#include "lmr_internal.h"

namespace lmr {

namespace {

constexpr int kMiThreads = 256;
constexpr double kFix = 4294967296.0;  // 2^32

// The windows and bin coordinates are evaluated in FP64: the gradient of MI
// sums products of windows and log-ratios that vary quickly with the bin
// coordinate, and FP32 coordinates (2^-24 of up to B) would move the step
// by ~1e-5 of its size.
__device__ __forceinline__ double bspline3(double t) {
  const double a = fabs(t);
  if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
  if (a < 2.0) {
    const double b = 2.0 - a;
    return b * b * b / 6.0;
  }
  return 0.0;
}
__device__ __forceinline__ double dbspline3(double t) {
  const double a = fabs(t), s = t < 0.0 ? -1.0 : 1.0;
  if (a < 1.0) return s * (-2.0 * a + 1.5 * a * a);
  if (a < 2.0) {
    const double b = 2.0 - a;
    return -s * 0.5 * b * b;
  }
  return 0.0;
}

// The four windows of bin coordinate c: bins k0 .. k0+3, k0 = floor(c) - 1.
__device__ __forceinline__ int windows(double c, double w[4]) {
  const double fl = floor(c);
  const int k0 = static_cast<int>(fl) - 1;
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] = bspline3(c - static_cast<double>(k0 + j));
  return k0;
}

template <typename T>
__global__ void __launch_bounds__(kMiThreads)
    k_mi_range(const T* __restrict__ F, const T* __restrict__ M, long long N,
               float* __restrict__ part) {
  float fl = INFINITY, fh = -INFINITY, ml = INFINITY, mh = -INFINITY;
  for (long long i = blockIdx.x * (long long)kMiThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kMiThreads) {
    const float f = ldf(F, static_cast<int>(i)), m = ldf(M, static_cast<int>(i));
    fl = fminf(fl, f);
    fh = fmaxf(fh, f);
    ml = fminf(ml, m);
    mh = fmaxf(mh, m);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    fl = fminf(fl, __shfl_xor(fl, off, 64));
    fh = fmaxf(fh, __shfl_xor(fh, off, 64));
    ml = fminf(ml, __shfl_xor(ml, off, 64));
    mh = fmaxf(mh, __shfl_xor(mh, off, 64));
  }
  __shared__ float red[4][kMiThreads / 64];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = fl;
    red[1][wv] = fh;
    red[2][wv] = ml;
    red[3][wv] = mh;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kMiThreads / 64; ++k) {
      red[0][0] = fminf(red[0][0], red[0][k]);
      red[1][0] = fmaxf(red[1][0], red[1][k]);
      red[2][0] = fminf(red[2][0], red[2][k]);
      red[3][0] = fmaxf(red[3][0], red[3][k]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[4 * blockIdx.x + q] = red[q][0];
  }
}

// map[0..3] = (lo_F, s_F, lo_M, s_M) with s = (B - 3) / (hi - lo) (FP64).
__global__ void k_mi_range_final(const float* __restrict__ part, int nblocks, int bins,
                                 double* __restrict__ map) {
  if (threadIdx.x != 0) return;
  float fl = INFINITY, fh = -INFINITY, ml = INFINITY, mh = -INFINITY;
  for (int b = 0; b < nblocks; ++b) {
    fl = fminf(fl, part[4 * b]);
    fh = fmaxf(fh, part[4 * b + 1]);
    ml = fminf(ml, part[4 * b + 2]);
    mh = fmaxf(mh, part[4 * b + 3]);
  }
  ml = fminf(ml, 0.0f);
  mh = fmaxf(mh, 0.0f);
  double df = static_cast<double>(fh) - fl, dm = static_cast<double>(mh) - ml;
  if (!(df > 0.0)) df = 1.0;
  if (!(dm > 0.0)) dm = 1.0;
  map[0] = fl;
  map[1] = (bins - 3) / df;
  map[2] = ml;
  map[3] = (bins - 3) / dm;
}

template <typename T>
__global__ void __launch_bounds__(kMiThreads)
    k_mi_hist(const T* __restrict__ F, const float* __restrict__ Mw, long long N, int bins,
              const double* __restrict__ map, unsigned long long* __restrict__ part,
              const DevState* __restrict__ st) {
  if (st && st->stalled) return;
  extern __shared__ unsigned long long h[];  // [waves][bins * bins]
  const int BB = bins * bins, nw = kMiThreads / 64, wv = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < nw * BB; k += kMiThreads) h[k] = 0ull;
  __syncthreads();
  const double flo = map[0], sf = map[1], mlo = map[2], sm = map[3];
  unsigned long long* hw = h + wv * BB;
  for (long long i = blockIdx.x * (long long)kMiThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kMiThreads) {
    double wa[4], wb[4];
    const int a0 = windows(1.0 + (static_cast<double>(ldf(F, static_cast<int>(i))) - flo) * sf,
                           wa);
    const int b0 = windows(1.0 + (static_cast<double>(Mw[i]) - mlo) * sm, wb);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = a0 + j;
      if (a < 0 || a >= bins || wa[j] == 0.0) continue;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int b = b0 + k;
        if (b < 0 || b >= bins || wb[k] == 0.0) continue;
        atomicAdd(&hw[a * bins + b],
                  static_cast<unsigned long long>(wa[j] * wb[k] * kFix + 0.5));
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < BB; k += kMiThreads) {
    unsigned long long s = 0ull;
    for (int w = 0; w < nw; ++w) s += h[w * BB + k];
    part[(long long)blockIdx.x * BB + k] = s;
  }
}

constexpr int kMiReduceThreads = 1024;

// One block.  p (FP64 [B*B]) and tab (FP64 [B*B], log2(p_ab / p_b), 0 where
// p_ab = 0) for the gradient; partials[0] = N MI (bits).
__global__ void __launch_bounds__(kMiReduceThreads)
    k_mi_reduce(const unsigned long long* __restrict__ part, int nblocks, int bins,
                long long N, double* __restrict__ p, double* __restrict__ tab,
                double* __restrict__ partials, const DevState* __restrict__ st) {
  if (st && st->stalled) return;
  const int BB = bins * bins;
  const double inv = 1.0 / (static_cast<double>(N) * kFix);
  for (int k = threadIdx.x; k < BB; k += kMiReduceThreads) {
    unsigned long long s = 0ull;
    for (int b = 0; b < nblocks; ++b) s += part[(long long)b * BB + k];
    p[k] = static_cast<double>(s) * inv;
  }
  __syncthreads();
  __shared__ double pa[64], pb[64];
  if (threadIdx.x < bins) {
    double sa = 0.0, sb = 0.0;
    for (int j = 0; j < bins; ++j) {
      sa += p[threadIdx.x * bins + j];
      sb += p[j * bins + threadIdx.x];
    }
    pa[threadIdx.x] = sa;
    pb[threadIdx.x] = sb;
  }
  __syncthreads();
  double mi = 0.0;
  for (int k = threadIdx.x; k < BB; k += kMiReduceThreads) {
    const double v = p[k];
    const int a = k / bins, b = k % bins;
    if (v > 0.0) {
      mi += v * log2(v / (pa[a] * pb[b]));
      tab[k] = log2(v / pb[b]);
    } else {
      tab[k] = 0.0;
    }
  }
  // fixed-order block sum of the per-thread terms
  __shared__ double red[kMiReduceThreads];
  red[threadIdx.x] = mi;
  __syncthreads();
  for (int w = kMiReduceThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[0] = red[0] * static_cast<double>(N);
}

template <typename T>
__global__ void __launch_bounds__(kMiThreads)
    k_mi_bwd(const T* __restrict__ F, const float* __restrict__ Mw, const float* dMw,
             long long N, int bins, const double* __restrict__ map,
             const double* __restrict__ tab, const DevState* __restrict__ st, float* graw) {
  if (st && (st->stalled || !st->accepted)) return;
  const double flo = map[0], sf = map[1], mlo = map[2], sm = map[3];
  for (long long i = blockIdx.x * (long long)kMiThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kMiThreads) {
    double wa[4];
    const int a0 = windows(1.0 + (static_cast<double>(ldf(F, static_cast<int>(i))) - flo) * sf,
                           wa);
    const double cm = 1.0 + (static_cast<double>(Mw[i]) - mlo) * sm;
    const int b0 = static_cast<int>(floor(cm)) - 1;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = a0 + j;
      if (a < 0 || a >= bins) continue;
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int b = b0 + k;
        if (b < 0 || b >= bins) continue;
        t += dbspline3(cm - static_cast<double>(b)) * tab[a * bins + b];
      }
      s += wa[j] * t;
    }
    const float d = static_cast<float>(-s * sm);  // -dMI/dMw (times N)
    const float n0 = dMw[i], n1 = dMw[N + i], n2 = dMw[2 * N + i];
    graw[i] = d * n0;
    graw[N + i] = d * n1;
    graw[2 * N + i] = d * n2;
  }
}

unsigned mi_blocks(long long N) {
  long long b = (N + kMiThreads * 8 - 1) / (kMiThreads * 8);
  if (b > kMiBlocks) b = kMiBlocks;
  return static_cast<unsigned>(b < 1 ? 1 : b);
}

}  // namespace

int mi_hist_blocks(long long N) { return static_cast<int>(mi_blocks(N)); }

hipError_t launch_mi_range(const void* F, const void* M, lmr_dtype t, const Geom& g, int bins,
                           float* part, double* map, hipStream_t s) {
  const unsigned nb = mi_blocks(g.N);
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_mi_range<uint16_t>, dim3(nb), dim3(kMiThreads), 0, s,
                       static_cast<const uint16_t*>(F), static_cast<const uint16_t*>(M), g.N,
                       part);
  else
    hipLaunchKernelGGL(k_mi_range<float>, dim3(nb), dim3(kMiThreads), 0, s,
                       static_cast<const float*>(F), static_cast<const float*>(M), g.N, part);
  hipLaunchKernelGGL(k_mi_range_final, dim3(1), dim3(64), 0, s, part, static_cast<int>(nb),
                     bins, map);
  return hipGetLastError();
}

hipError_t launch_mi_fwd(const void* F, lmr_dtype t, const float* Mw, const Geom& g, int bins,
                         const double* map, unsigned long long* hpart, double* p, double* tab,
                         double* partials, const DevState* st, hipStream_t s) {
  const unsigned nb = mi_blocks(g.N);
  const size_t lds = sizeof(unsigned long long) * (kMiThreads / 64) * bins * bins;
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_mi_hist<uint16_t>, dim3(nb), dim3(kMiThreads), lds, s,
                       static_cast<const uint16_t*>(F), Mw, g.N, bins, map, hpart, st);
  else
    hipLaunchKernelGGL(k_mi_hist<float>, dim3(nb), dim3(kMiThreads), lds, s,
                       static_cast<const float*>(F), Mw, g.N, bins, map, hpart, st);
  hipLaunchKernelGGL(k_mi_reduce, dim3(1), dim3(kMiReduceThreads), 0, s, hpart,
                     static_cast<int>(nb), bins, g.N, p, tab, partials, st);
  return hipGetLastError();
}

hipError_t launch_mi_bwd(const void* F, lmr_dtype t, const float* Mw, const float* dMw,
                         const Geom& g, int bins, const double* map, const double* tab,
                         const DevState* st, float* graw, hipStream_t s) {
  const unsigned nb = static_cast<unsigned>(std::min<long long>((g.N + 255) / 256, 4096));
  if (t == LMR_BF16)
    hipLaunchKernelGGL(k_mi_bwd<uint16_t>, dim3(nb), dim3(kMiThreads), 0, s,
                       static_cast<const uint16_t*>(F), Mw, dMw, g.N, bins, map, tab, st,
                       graw);
  else
    hipLaunchKernelGGL(k_mi_bwd<float>, dim3(nb), dim3(kMiThreads), 0, s,
                       static_cast<const float*>(F), Mw, dMw, g.N, bins, map, tab, st, graw);
  return hipGetLastError();
}

}  // namespace lmr
