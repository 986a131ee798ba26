/*
 * lmreg learned initializer — a small 3D U-Net that predicts an initial
 * displacement field from a (fixed, moving) pair; the factored LM method then
 * refines from it and remains the fallback when the prediction loses.
 *
 * The network (four resolution levels with 16/32/64/128 channels, two 3x3x3
 * convolutions per level with ReLU, 2x2x2 average pooling down, x2 nearest
 * upsampling up with skip concatenation, a final 3x3x3 convolution to the 3
 * field components) is defined layer by layer below.  Convolutions run on
 * the MFMA matrix cores with BF16 operands and FP32 accumulation; master
 * weights, gradients and Adam moments are FP32.  Training targets are fields
 * the LM method converged to, so the network learns to start the iteration
 * close to where it ends.
 *
 * Layers (index: input -> output, channels), d = level (resolution / 2^d):
 *   0: input (F, M)        -> e1a  2 -> 16    d0     1: e1a -> e1 16 -> 16  d0
 *   2: pool(e1)            -> e2a 16 -> 32    d1     3: e2a -> e2 32 -> 32  d1
 *   4: pool(e2)            -> e3a 32 -> 64    d2     5: e3a -> e3 64 -> 64  d2
 *   6: pool(e3)            -> e4a 64 -> 128   d3     7: e4a -> e4 128->128  d3
 *   8: [up(e4), e3]        -> f3a 192 -> 64   d2     9: f3a -> f3 64 -> 64  d2
 *  10: [up(f3), e2]        -> f2a 96 -> 32    d1    11: f2a -> f2 32 -> 32  d1
 *  12: [up(f2), e1]        -> f1a 48 -> 16    d0    13: f1a -> f1 16 -> 16  d0
 *  14: f1                  -> field 16 -> 3   d0    (no ReLU)
 * Parameters: one flat FP32 vector, per layer W [27][cin][cout] (tap
 * t = 9 (dz+1) + 3 (dy+1) + (dx+1) reads the input at v + (dx, dy, dz)) then
 * b [cout], layers in index order.
 *
 * Conventions as in lmreg.h (device pointers are caller-owned, work is
 * enqueued on the network's stream, statuses instead of exceptions).
 */
#ifndef LMREG_UNET_H
#define LMREG_UNET_H

#include "lmreg.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LMR_UNET_LAYERS 15

typedef struct lmr_unet lmr_unet;

/* Total number of FP32 parameters. */
int64_t lmr_unet_param_count(void);
/* Shape of layer `layer`: input and output channels, ReLU flag and the offset
 * of its W in the flat parameter vector (b follows W).  LMR_EINVAL if out of
 * range. */
lmr_status lmr_unet_layer_info(int layer, int* cin, int* cout, int* relu, int64_t* offset);

/* A network working at nz x ny x nx voxels (each divisible by 8, product
 * < 2^28), bound to `stream`.  Allocates parameters (zero), gradients, Adam
 * moments, BF16 weight packs and every activation and gradient buffer (about
 * 700 bytes per voxel); no later call allocates.  LMR_EINVAL, LMR_ENOMEM. */
lmr_status lmr_unet_create(lmr_unet** out, int nz, int ny, int nx, hipStream_t stream);
void lmr_unet_destroy(lmr_unet* net);

/* Copies params (device, lmr_unet_param_count floats) into the network and
 * resets the Adam moments and step count.  Asynchronous. */
lmr_status lmr_unet_set_params(lmr_unet* net, const float* params);
/* Copy out the parameters / the accumulated gradients (device arrays). */
lmr_status lmr_unet_get_params(lmr_unet* net, float* params);
lmr_status lmr_unet_get_grads(lmr_unet* net, float* grads);

/* Forward pass.  fixed, moving: device images of type img, of the network's
 * size (pool = 0) or of twice its size in every dimension (pool = 1: they are
 * average-pooled by 2 first, as the learned initializer does for full-
 * resolution pairs).  field (device [3][nz][ny][nx] FP32, may be NULL)
 * receives the predicted displacement (x, y, z components, voxels of the
 * network's grid).  Keeps the activations for lmr_unet_backward. */
lmr_status lmr_unet_forward(lmr_unet* net, const void* fixed, const void* moving,
                            lmr_dtype img, int pool, float* field);

/* Backward pass of the mean squared error between the last forward output
 * and target_scale * target (target: device [3][nz][ny][nx]), averaged over
 * all 3 nz ny nx values.  Gradients of every parameter are written
 * (accumulate = 0) or added (accumulate = 1, for mini-batches); loss (device
 * double, may be NULL) receives the MSE.  LMR_ESTATE without a preceding
 * lmr_unet_forward. */
lmr_status lmr_unet_backward(lmr_unet* net, const float* target, double target_scale,
                             int accumulate, double* loss);

/* One Adam step on the FP32 master parameters with the accumulated gradients
 * times grad_scale (e.g. 1 / mini-batch size); bias-corrected moments; the
 * BF16 packs are refreshed.  lr > 0, 0 <= beta1, beta2 < 1, eps > 0. */
lmr_status lmr_unet_adam(lmr_unet* net, double lr, double beta1, double beta2,
                         double eps, double grad_scale);

/* Test hook: layer `layer` alone, with the network's current (BF16-packed)
 * weights, on the grid of the layer's level (dims >> level).  Checks each
 * convolution of the forward and backward passes element by element.
 *   x   device BF16 bits, channels last [N_l][ldx] (ldx >= cin, a multiple of
 *       4, 8-byte aligned; channels cin..round4(cin)-1 must be finite);
 *   y   (may be NULL) device FP32 [N_l][ldy], ldy >= cout: receives
 *       act(conv(x) + b) before any rounding (act = ReLU except the head);
 *   dz  (may be NULL) device BF16 [N_l][ldz] (ldz >= cout, a multiple of 4,
 *       8-byte aligned): a gradient of the pre-activation output; then dW
 *       [27][cin][cout] and db [cout] (device FP32) receive the parameter
 *       gradients and dx (may be NULL; device BF16 [N_l][lddx], lddx >= cin)
 *       the input gradient.
 * The network's own activations and gradients are not touched.  Enqueues
 * only.  LMR_EINVAL on a bad layer, pointer or stride. */
lmr_status lmr_unet_layer_probe(lmr_unet* net, int layer, const uint16_t* x, int ldx,
                                float* y, int ldy, const uint16_t* dz, int ldz,
                                uint16_t* dx, int lddx, float* dW, float* db);

#ifdef __cplusplus
}
#endif
#endif /* LMREG_UNET_H */
