/*
 * lbm_cnn.h - kernels of the learned coarse-grid correction (single GPU).
 *
 * The paper defines no closure; this is the network the correction uses: 3x3
 * convolutions with periodic (circular) padding on [batch][channel][y][x]
 * FP32 activations,
 *
 *   Y[b][co][y][x] = bias[co] + sum_{ci, dy, dx} W[co][ci][dy+1][dx+1] X[b][ci][y+dy][x+dx]
 *
 * (indices mod h, w), computed on BF16 matrix cores (operands rounded to BF16,
 * FP32 accumulation).  Weights are kept in FP32 by the caller and packed to the
 * BF16 operand layout with lbm_conv_pack before use.  All pointers are device
 * pointers unless stated; every call is enqueued on `stream` (hipStream_t as
 * void*) and is asynchronous unless stated.  Limits: w a multiple of 64,
 * cin and cout in 1..64.
 */
#ifndef LBM_CNN_H
#define LBM_CNN_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of the packed BF16 weight operand of a cin -> cout layer. */
size_t lbm_conv_packed_bytes(int32_t cin, int32_t cout);

/* Pack W[cout][cin][3][3] (FP32) into `packed`.  transpose != 0 packs instead
 * the weights of the input-gradient convolution of that layer (a cout -> cin
 * convolution with W'[ci][co][tap] = W[co][ci][8 - tap], taps flipped), so
 * that dX = conv(dY, W') with no bias. */
lbm_status lbm_conv_pack(const float* w, int32_t cin, int32_t cout, int32_t transpose, void* packed,
                         void* stream);

#define LBM_CONV_RELU 0x1u /* apply max(0, .) after the bias */

/* Y = conv(X, W) + bias (bias may be NULL), then ReLU if flags & LBM_CONV_RELU,
 * then, if mask != NULL, Y *= (mask > 0) elementwise (mask has Y's shape; used
 * for the ReLU derivative in the backward pass).  x: [batch][cin][h][w],
 * y: [batch][cout][h][w]; x and y must not overlap. */
lbm_status lbm_conv_forward(const float* x, int32_t batch, int32_t cin, int32_t h, int32_t w,
                            const void* packed, int32_t cout, const float* bias, const float* mask,
                            uint32_t flags, float* y, void* stream);

/* Inference of the whole correction network in one launch, for 2D moment
 * planes m[3][h][w] (rho, q_x, q_y; FP32):
 *   x = ((rho - rho_ref)/s_rho, (q_x/rho)/s_u, (q_y/rho)/s_u)   (as lbm_closure_features)
 *   y = L4(relu(L3(relu(L2(relu(L1(x)))))))   channels 3 -> 32 -> 32 -> 32 -> 3
 * where L_l is the 3x3 periodic convolution of lbm_conv_forward with the
 * forward-packed operand packed[l] (lbm_conv_pack, transpose = 0) and the
 * bias bias[l]; packed and bias are host arrays of 4 device pointers.  The
 * result equals the four lbm_conv_forward calls bit for bit; the activations
 * never leave the chip.  y: [3][h][w] FP32.  partials receives, for each
 * 16 x 16 tile t (row-major over the tiles), the FP64 sums of the tile's
 * three output channels in partials[4t .. 4t+2] (partials[4t+3] = 0);
 * lbm_net_partials_bytes(h, w) bytes.  h and w: positive multiples of 16;
 * s_rho, s_u > 0.  Returns LBM_EINVAL otherwise. */
size_t lbm_net_partials_bytes(int32_t h, int32_t w);
lbm_status lbm_net_infer(const float* moments, int32_t h, int32_t w, double rho_ref, float s_rho,
                         float s_u, const void* const* packed, const float* const* bias, float* y,
                         double* partials, void* stream);

/* Scratch bytes for lbm_conv_wgrad. */
size_t lbm_conv_wgrad_scratch_bytes(int32_t batch, int32_t cin, int32_t cout, int32_t h, int32_t w);

/* Weight and bias gradients of Y = conv(X, W) + b given dL/dY:
 *   dw[co][ci][tap] = sum_{b,y,x} dy[b][co][y][x] X[b][ci][y+dy][x+dx],  db[co] = sum dy[b][co]
 * Deterministic: per-block partials in `scratch`, then a fixed-order sum. */
lbm_status lbm_conv_wgrad(const float* x, const float* dy, int32_t batch, int32_t cin, int32_t cout,
                          int32_t h, int32_t w, float* dw, float* db, void* scratch, void* stream);

/* grad = 2 (out - target) / n; *loss_dev (device double) = mean((out - target)^2).
 * scratch: at least lbm_reduce_scratch_bytes(n) bytes. */
size_t lbm_reduce_scratch_bytes(int64_t n);
lbm_status lbm_mse(const float* out, const float* target, int64_t n, float* grad, double* loss_dev,
                   void* scratch, void* stream);

/* Adam step (bias-corrected, step number t >= 1) on n FP32 parameters:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps). */
lbm_status lbm_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                    float eps, int32_t t, void* stream);

/* Root mean square of each of `channels` consecutive planes of n values:
 * out_dev[c] = sqrt(mean(x[c][:]^2)) (device doubles).  scratch as for lbm_mse. */
lbm_status lbm_channel_rms(const float* x, int32_t channels, int64_t n, double* out_dev, void* scratch,
                           void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_CNN_H */
