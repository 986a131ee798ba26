// lmr_loss_grad_noalloc: the loss and gradients of a field (lmr_loss_grad)
// without a context and without any device allocation, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its workspace is one static device
// array of this library; each GPU the library runs on holds its own copy
// from module load until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.h"
#include "lmr_internal.h"

namespace {

constexpr long long kMaxVoxels = 1LL << 20;  // largest volume a call accepts
constexpr long long kMaxParts = 1LL << 17;   // FP64 partials of the forward pass

// Workspace layout (byte offsets, each a multiple of 256):
//   window mean and variance of F  FP64 [2][N]
//   the four LNCC adjoint maps     FP32 [4][N]
//   warped moving image            FP32 [N]
//   raw gradient (when the caller  FP32 [3][N]
//     asks only for the smoothed one)
//   forward partials               FP64 [kMaxParts]
//   pair state read by the decision kernel
constexpr size_t kOffMaps = 16 * kMaxVoxels;
constexpr size_t kOffMw = kOffMaps + 16 * kMaxVoxels;
constexpr size_t kOffGraw = kOffMw + 4 * kMaxVoxels;
constexpr size_t kOffParts = kOffGraw + 12 * kMaxVoxels;
constexpr size_t kOffState = kOffParts + 8 * kMaxParts;
constexpr size_t kScratchBytes = kOffState + ((sizeof(lmr::DevState) + 255) / 256) * 256;

}  // namespace

// The workspace.  In host code this name is a host-side stand-in, not a
// device address: the device address is obtained once per device with
// hipGetSymbolAddress and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of the workspace on the current device (looked up on the
// first call per device, with that device current).
lmr_status scratch_of_current_device(char** out) {
  int dev = 0;
  LMR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return LMR_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    LMR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return LMR_OK;
}

}  // namespace

extern "C" lmr_status lmr_loss_grad_noalloc(const void* F, const void* M, lmr_dtype img,
                                            const float* u, int nz, int ny, int nx,
                                            const lmr_params* p, double* loss_dev,
                                            float* g_raw, float* g_smooth, float* cc_map,
                                            hipStream_t stream) {
  using namespace lmr;
  if (!F || !M || !u || !loss_dev || !params_ok(p)) return LMR_EINVAL;
  if (img != LMR_F32 && img != LMR_BF16) return LMR_EINVAL;
  if (nz < 1 || ny < 1 || nx < 1 || nz > 65535) return LMR_EINVAL;
  if (g_raw && g_raw == g_smooth) return LMR_EINVAL;
  const long long N = (long long)nz * ny * nx;
  if (N > kMaxVoxels) return LMR_EINVAL;  // beyond the static workspace
  const Geom g{nz, ny, nx, N};
  const int nparts = fwd_num_blocks(g, *p);
  if (nparts > kMaxParts) return LMR_EINVAL;
  char* base = nullptr;
  const lmr_status st = scratch_of_current_device(&base);
  if (st != LMR_OK) return st;
  double* fstat = reinterpret_cast<double*>(base);
  float* maps = reinterpret_cast<float*>(base + kOffMaps);
  float* Mw = reinterpret_cast<float*>(base + kOffMw);
  float* graw = reinterpret_cast<float*>(base + kOffGraw);
  double* parts = reinterpret_cast<double*>(base + kOffParts);
  DevState* dst = reinterpret_cast<DevState*>(base + kOffState);
  // every workspace value a kernel reads here was written earlier in the
  // same call (statistics, warp, maps, one partial per forward tile); the
  // decision kernel in probe mode reads the pair state but uses none of it
  const DecideParams dp{p->lambda_inc, p->lambda_dec, p->lambda_min, p->lambda_max, p->tau,
                        p->max_retries};
  LMR_HIP(launch_fstat(F, img, g, *p, fstat, stream));
  LMR_HIP(launch_warp(M, img, u, g, Mw, nullptr, stream));
  LMR_HIP(launch_fwd(F, img, Mw, fstat, g, *p, nullptr, maps, parts, nparts, cc_map, stream));
  LMR_HIP(launch_decide(dst, parts, nparts, N, dp, 2, -1, 0.0, loss_dev, stream));
  if (g_raw || g_smooth) {
    float* gr = g_raw ? g_raw : graw;
    LMR_HIP(launch_bwd(F, M, img, Mw, maps, g, *p, nullptr, nullptr, nullptr, u, nullptr,
                       gr, stream));
    if (g_smooth) LMR_HIP(launch_smooth(gr, g, *p, nullptr, g_smooth, stream));
  }
  return LMR_OK;
}
