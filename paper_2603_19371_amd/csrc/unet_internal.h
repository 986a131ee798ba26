// Launchers of the U-Net kernels (k_unet.hip), used by api_unet.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lmreg.h"

namespace lmr {

// A 3x3x3 convolution (zero padding 1) of a channels-last BF16 tensor.
//   X: input, element (v, c) at X[v*ldx + c]; channels [0, cin_valid) are used
//      and the 4-channel group holding cin_valid-1 is read whole (the
//      channels of that group past cin_valid must be finite).
//   W: packed BF16 weights [27][cout_p][cin_p].
//   bias (FP32, may be NULL), relu: epilogue y = act(acc + bias).
//   Y (BF16, may be NULL) and yf (FP32, may be NULL): outputs, stride ldy / ldf.
// Requirements (checked by the caller): ldx, and the element offset of X, are
// multiples of 4; cin_p, cout_p multiples of 16.
struct ConvArgs {
  const uint16_t* X;
  int ldx, cin_valid, cin_p;
  const uint16_t* W;
  const float* bias;
  int cout, cout_p;
  uint16_t* Y;
  int ldy;
  float* yf;
  int ldf;
  int nz, ny, nx;
  int relu;
};
hipError_t unet_conv(const ConvArgs& a, hipStream_t s);

// Weight and bias gradients of a convolution from its input X and the
// gradient dZ of its pre-activation output:
//   dW[t][ci][co] = sum_v X[v + d_t, ci] dZ[v, co],  db[co] = sum_v dZ[v, co]
// written unpadded ([27][cin][cout], [cout], FP32; accumulate = 1 adds to
// dW, db).  `part` and `partb` are
// workspaces of unet_wgrad_part_floats / unet_wgrad_bias_floats floats.
// X and dZ: channel strides and element offsets multiples of 4 (8-byte items).
long long unet_wgrad_part_floats(int cin_p, int cout_p, int nz, int ny, int nx);
long long unet_wgrad_bias_floats(int cin_p, int cout_p, int nz, int ny, int nx);
hipError_t unet_wgrad(const uint16_t* X, int ldx, int cin, int cin_p, const uint16_t* dZ,
                      int ldz, int cout, int cout_p, int nz, int ny, int nx, float* part,
                      float* partb, float* dW, float* db, int accumulate, hipStream_t s);

// d[v, c] = 0 where a[v, c] <= 0 (gradient through a ReLU), c < C.
hipError_t unet_relu_mask(uint16_t* d, int ldd, const uint16_t* a, int lda, int C,
                          long long N, hipStream_t s);
// 2x2x2 average pooling (fine dims nz, ny, nx) and its gradient (add: add
// into dX instead of overwriting).
hipError_t unet_pool2(const uint16_t* X, int ldx, int C, int nz, int ny, int nx,
                      uint16_t* Y, int ldy, hipStream_t s);
hipError_t unet_pool2_back(const uint16_t* dY, int ldy, int C, int nz, int ny, int nx,
                           uint16_t* dX, int ldx, int add, hipStream_t s);
// x2 nearest upsampling to fine dims (nz, ny, nx) and its gradient.
hipError_t unet_up2(const uint16_t* X, int ldx, int C, int nz, int ny, int nx, uint16_t* Y,
                    int ldy, hipStream_t s);
hipError_t unet_up2_back(const uint16_t* dY, int ldy, int C, int nz, int ny, int nx,
                         uint16_t* dX, int ldx, int add, hipStream_t s);
// Network input X [N][4] = (F, M, 0, 0) at dims (nz, ny, nx); pool = 1 reads
// images of twice the size and average-pools them by 2.
hipError_t unet_input(const void* F, const void* M, lmr_dtype t, int nz, int ny, int nx,
                      int pool, uint16_t* X, hipStream_t s);
// Planar field [3][N] from the FP32 head output (stride ldf).
hipError_t unet_head_to_field(const float* yf, int ldf, long long N, float* field,
                              hipStream_t s);
// MSE against target*tscale (planar [3][N]); dout (BF16, stride ld) receives
// the gradient and *loss (device) the mean squared error.  part: workspace of
// unet_mse_blocks(N) doubles.
int unet_mse_blocks(long long N);
hipError_t unet_mse(const float* yf, int ldf, const float* target, float tscale,
                    long long N, uint16_t* dout, int ld, double* part, double* loss,
                    hipStream_t s);
hipError_t unet_zero(uint16_t* p, long long n, hipStream_t s);
hipError_t unet_adam(float* p, float* m, float* v, const float* g, long long n, float lr,
                     float b1, float b2, float eps, float c1, float c2, float gscale,
                     hipStream_t s);
// W [27][cin][cout] FP32 -> Wf [27][cout_p][cin_p] and the tap-reversed,
// transposed Wb [27][cin_p][cout_p] (BF16, zero padded).
hipError_t unet_pack(const float* W, int cin, int cout, int cin_p, int cout_p,
                     uint16_t* Wf, uint16_t* Wb, hipStream_t s);

}  // namespace lmr
