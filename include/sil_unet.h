/*
 * sil_unet.h -- gfx950 kernels of the U-Net trained on the auto-labels
 * (arXiv 2403.13135, section III-C "U-Net Model for Sea-Ice Classification":
 * two 3x3 convolutions with ReLU per level, 2x2 max pooling with stride 2,
 * 2x2 up-convolutions that halve the channels, concatenation with the skip
 * map, a 1x1 convolution to the 3 classes; "U-Net Training": categorical
 * cross-entropy and the Adam optimizer).  The network these kernels serve
 * adds batch normalisation after each 3x3 convolution and uses "same"
 * padding.
 *
 * Conventions:
 *   - Activations are bf16, NHWC, contiguous ([N][H][W][C]); a "pixel" is one
 *     (n, h, w); P = N*H*W.  Weights used by the convolutions are bf16; master
 *     weights, gradients, statistics and the loss are fp32.
 *   - 3x3 and up-convolutions run on MFMA (v_mfma_f32_16x16x32_bf16) with fp32
 *     accumulation; all other steps are plain HIP kernels.
 *   - Channel counts must be multiples of 8 (pad the 3-channel input to 8
 *     with zeros); batch-norm and head channel counts must divide 256.
 *     Violations: SIL_EINVAL.  Tensors are read and written in 16-byte
 *     chunks, so their base addresses must be 16-byte aligned (any device
 *     allocation is).
 *   - Every call is asynchronous on `stream` (hipStream_t or NULL), allocates
 *     nothing and validates its sizes before enqueueing.  Outputs marked
 *     "accumulate" are ADDED to (zero them first, e.g. sil_unet_fill_f32).
 *   - Returns SIL_OK, SIL_EINVAL (NULL pointer, non-positive or unsupported
 *     size) or SIL_EDEVICE (launch failure).
 */
#ifndef SIL_UNET_H
#define SIL_UNET_H

#include <stdint.h>

#include "sil.h"

#ifdef __cplusplus
extern "C" {
#endif

/* 3x3 convolution, stride 1, zero padding 1, no bias.  The input is the
 * channel concatenation of x0 [N][H][W][c0] and x1 [N][H][W][c1] (x1 NULL and
 * c1 = 0 for a single input).  w: [cout][3][3][c0+c1].  y: [N][H][W][cout].
 * stats (nullable, fp32 [2][cout], accumulate): per-channel sum and sum of
 * squares of the fp32 outputs before rounding to bf16. */
int sil_unet_conv3x3(const void* x0, int32_t c0, const void* x1, int32_t c1, const void* w,
                     void* y, float* stats, int32_t N, int32_t H, int32_t W, int32_t cout,
                     void* stream);

/* Inference form of a conv + batch-norm + ReLU layer: the same 3x3
 * convolution as sil_unet_conv3x3, with y = max(0, conv * scale[co] +
 * shift[co]) applied to the fp32 result before rounding to bf16 (batch norm
 * with running statistics folded into scale/shift, fp32 [cout]).  Every output
 * pixel depends only on its own input neighbourhood, so a chip's result does
 * not depend on the rest of the batch. */
int sil_unet_conv3x3_affine_relu(const void* x0, int32_t c0, const void* x1, int32_t c1,
                                 const void* w, const float* scale, const float* shift, void* y,
                                 int32_t N, int32_t H, int32_t W, int32_t cout, void* stream);

/* Batch-norm backward sums of a conv + batch-norm + ReLU layer, formed by the
 * call that produces the gradient dout of that layer's output (passed to the
 * input-gradient, pooling and head backward calls below; NULL: none).  With d
 * = dout where the layer's ReLU passed (xhat * gamma + beta > 0, xhat = (z -
 * mean) * rstd) and 0 elsewhere: sum_d[c] += sum_p d (the beta gradient),
 * sum_dxhat[c] += sum_p d * xhat (the gamma gradient), both fp32 [C]
 * accumulate; sil_unet_bn_relu_bwd_apply then forms dz from them.  z: the
 * layer's batch-norm input [P][C] bf16, same pixels as dout; mr: its (mean,
 * rstd) [2][C].  C must equal dout's channel count and 256 % (C/8) == 0. */
typedef struct sil_unet_bn_grad {
  const void* z;
  const float* mr;
  const float* gamma;
  const float* beta;
  float* sum_d;
  float* sum_dxhat;
  int32_t C;
} sil_unet_bn_grad;

/* Input gradient of sil_unet_conv3x3: dx = conv3x3(dy, wt) with wt the
 * flipped, transposed weights [c0+c1][3][3][cout] (sil_unet_flip3x3).  The
 * result is split by channel into dx0 [N][H][W][c0] and dx1 [..][c1]
 * (dx1 NULL when c1 = 0).  bn (nullable, only with c1 = 0): the sums of the
 * layer whose output gradient dx0 is. */
int sil_unet_conv3x3_dgrad(const void* dy, int32_t cout, const void* wt, void* dx0, int32_t c0,
                           void* dx1, int32_t c1, int32_t N, int32_t H, int32_t W,
                           const sil_unet_bn_grad* bn, void* stream);

/* Weight gradient of sil_unet_conv3x3 (accumulate): dw [cout][3][3][c0+c1] fp32
 * += sum over pixels of dy (x) im2col(concat(x0, x1)). */
int sil_unet_conv3x3_wgrad(const void* dy, int32_t cout, const void* x0, int32_t c0,
                           const void* x1, int32_t c1, float* dw, int32_t N, int32_t H,
                           int32_t W, void* stream);

/* wt[ci][r][s][co] = w[co][2-r][2-s][ci] (bf16). */
int sil_unet_flip3x3(const void* w, void* wt, int32_t cout, int32_t cin, void* stream);

/* 2x2 up-convolution, stride 2 (transposed convolution): y[n][2h+i][2w+j][co]
 * = b[co] + sum_ci x[n][h][w][ci] * w[i][j][co][ci].  x [N][H][W][cin],
 * w bf16 [2][2][cout][cin], b fp32 [cout], y [N][2H][2W][cout]. */
int sil_unet_upconv(const void* x, const void* w, const float* b, void* y, int32_t N, int32_t H,
                    int32_t W, int32_t cin, int32_t cout, void* stream);

/* Input gradient: dx[n][h][w][ci] = sum_{i,j,co} dy[n][2h+i][2w+j][co] *
 * w[i][j][co][ci], with wt = the weights as [ci][2][2][co] (sil_unet_up_t).
 * bn (nullable): the sums of the layer whose output gradient dx is. */
int sil_unet_upconv_dgrad(const void* dy, const void* wt, void* dx, int32_t N, int32_t H,
                          int32_t W, int32_t cin, int32_t cout, const sil_unet_bn_grad* bn,
                          void* stream);

/* Weight and bias gradients (accumulate): dw fp32 [2][2][cout][cin],
 * db fp32 [cout]. */
int sil_unet_upconv_wgrad(const void* x, const void* dy, float* dw, float* db, int32_t N,
                          int32_t H, int32_t W, int32_t cin, int32_t cout, void* stream);

/* wt[ci][i][j][co] = w[i][j][co][ci] (bf16). */
int sil_unet_up_t(const void* w, void* wt, int32_t cin, int32_t cout, void* stream);

/* Batch normalisation with batch statistics and ReLU:
 * out = max(0, (z - mean) * rstd * gamma + beta), mean and biased variance from
 * stats ([2][C]: sums over `count` values), rstd = 1/sqrt(var + eps).  Writes
 * mr [2][C] = (mean, rstd) for the backward pass. */
int sil_unet_bn_relu(const void* z, const float* stats, const float* gamma, const float* beta,
                     float eps, int64_t count, void* out, float* mr, int64_t P, int32_t C,
                     void* stream);

/* Inference-mode batch normalisation and ReLU with fixed per-channel scale and
 * shift (scale = gamma/sqrt(running_var + eps), shift = beta - running_mean *
 * scale): out = max(0, z * scale + shift).  Each pixel's result depends only on
 * that pixel, so outputs do not depend on what else is in the batch. */
int sil_unet_affine_relu(const void* z, const float* scale, const float* shift, void* out,
                         int64_t P, int32_t C, void* stream);

/* Backward of sil_unet_bn_relu.  dout, z: [P][C] bf16; writes dz [P][C] bf16.
 * With red (caller-provided fp32 [2][C] scratch, zeroed by the call) non-NULL,
 * dgamma and dbeta (fp32 [C]) accumulate.  With red NULL the per-channel sums
 * are formed in dbeta and dgamma themselves, which must then hold zeros on
 * entry (a fresh gradient), and the call makes no separate fill or add
 * launch. */
int sil_unet_bn_relu_bwd(const void* dout, const void* z, const float* mr, const float* gamma,
                         const float* beta, void* dz, float* dgamma, float* dbeta, float* red,
                         int64_t P, int32_t C, void* stream);

/* The second half of sil_unet_bn_relu_bwd, with the per-channel sums given
 * (sum_d = the beta gradient, sum_dxhat = the gamma gradient, e.g. formed
 * through a sil_unet_bn_grad request): dz = gamma * rstd * (d - (sum_d + xhat
 * sum_dxhat) / P). */
int sil_unet_bn_relu_bwd_apply(const void* dout, const void* z, const float* mr,
                               const float* gamma, const float* beta, const float* sum_d,
                               const float* sum_dxhat, void* dz, int64_t P, int32_t C,
                               void* stream);

/* 2x2 max pooling, stride 2 (H, W even).  idx [N][H/2][W/2][C] u8 records
 * the winning position (first maximum in row-major window order). */
int sil_unet_maxpool(const void* x, void* y, uint8_t* idx, int32_t N, int32_t H, int32_t W,
                     int32_t C, void* stream);
/* Backward: dx [N][H][W][C] = dy routed to each window's winner (zero
 * elsewhere), plus dadd [N][H][W][C] when non-NULL (the gradient the same
 * tensor receives from its other consumer, e.g. the skip connection; summed in
 * fp32, rounded once to bf16).  dadd may be dx itself.  bn (nullable): the
 * sums of the layer whose output gradient dx is. */
int sil_unet_maxpool_bwd(const void* dy, const uint8_t* idx, const void* dadd, void* dx,
                         int32_t N, int32_t H, int32_t W, int32_t C, const sil_unet_bn_grad* bn,
                         void* stream);

/* 1x1 head: logits[p][k] = b[k] + sum_c x[p][c] w[k][c], k < 3 (fp32 out). */
int sil_unet_head(const void* x, const float* w, const float* b, float* logits, int64_t P,
                  int32_t C, void* stream);

/* Softmax cross-entropy over 3 classes: loss[0] += scale * sum_p -log
 * softmax(l_p)[y_p] (accumulate; scale = 1/P gives the mean);
 * dlogits[p] = (softmax(l_p) - onehot(y_p)) * scale.
 * labels: u8 [P] in 0..2; dlogits nullable. */
int sil_unet_softmax_xent(const float* logits, const uint8_t* labels, float* loss,
                          float* dlogits, float scale, int64_t P, void* stream);

/* The head and the softmax cross-entropy in one pass (section III-C): per
 * pixel the logits of sil_unet_head, then the loss and dlogits of
 * sil_unet_softmax_xent, with the same arithmetic (identical dlogits and
 * logits).  loss[0] accumulates; logits (fp32 [P][3]) is nullable: written
 * only when given.  labels u8 [P] in 0..2. */
int sil_unet_head_xent(const void* x, const float* w, const float* b, const uint8_t* labels,
                       float* loss, float* dlogits, float* logits, float scale, int64_t P,
                       int32_t C, void* stream);

/* Head backward: with d = dlogits * dscale[0] (dscale: nullable device fp32
 * scalar, the gradient arriving at the loss; NULL means 1), dx [P][C] bf16 =
 * d w; dw fp32 [3][C] += sum_p d x; db fp32 [3] += sum_p d.  bn (nullable):
 * the sums of the layer whose output gradient dx is. */
int sil_unet_head_bwd(const void* x, const float* w, const float* dlogits, const float* dscale,
                      void* dx, float* dw, float* db, int64_t P, int32_t C,
                      const sil_unet_bn_grad* bn, void* stream);

/* Class map: labels[p] = argmax_k logits[p][k] (first maximum). */
int sil_unet_argmax(const float* logits, uint8_t* labels, int64_t P, void* stream);

/* Write the class map of chips back into a scene label plane: for chip n with
 * origin (origins[2n], origins[2n+1]), labels[y0+h][x0+w] = argmax_k
 * logits[n][h][w][k] for pixels inside the H x W scene.  logits fp32
 * [n_chips][chip][chip][3]; labels [H][lpitch]. */
int sil_unet_scatter_argmax(const float* logits, const int32_t* origins, int32_t n_chips,
                            int32_t chip, uint8_t* labels, int32_t H, int32_t W, int64_t lpitch,
                            void* stream);

/* Network input from a planar 16-bit scene [3][H][pitch] (bands B2, B3, B4):
 * for chip n with origin (y0, x0) = (origins[2n], origins[2n+1]) (device int32),
 * out[n][h][w][c] = bf16(scene[c][y0+h][x0+w] * inv_refl) for c < 3 and 0 for
 * c in 3..7; pixels outside the scene are 0.  out: [n_chips][chip][chip][8]. */
int sil_unet_chips_input(const uint16_t* scene, int32_t H, int32_t W, int64_t pitch,
                         const int32_t* origins, int32_t n_chips, int32_t chip, float inv_refl,
                         void* out, void* stream);

/* Adam (Kingma & Ba) with bias correction on fp32 master weights; writes the
 * bf16 copy when wbf is non-NULL.  m, v: fp32 moments. */
int sil_unet_adam(float* w, const float* g, float* m, float* v, void* wbf, int64_t n, float lr,
                  float beta1, float beta2, float eps, int32_t step, void* stream);

/* One tensor of a multi-tensor Adam step: w (fp32 master weights), g
 * (gradient), m, v (fp32 moments), n elements each. */
typedef struct sil_unet_adam_tensor {
  float* w;
  const float* g;
  float* m;
  float* v;
  int64_t n;
} sil_unet_adam_tensor;

/* sil_unet_adam's update (without the bf16 copy) on `count` tensors in one
 * launch per 64 tensors.  The step number (>= 1) is `step`, or, when step_dev
 * (a device int32) is non-NULL, the value it holds when the kernel runs: a
 * launch captured in a graph then takes the step current at each replay (the
 * caller advances it, e.g. with sil_unet_counter_add in the same graph).  The
 * bias corrections 1 - beta^step are formed on the device. */
int sil_unet_adam_multi(const sil_unet_adam_tensor* t, int32_t count, float lr, float beta1,
                        float beta2, float eps, int32_t step, const int32_t* step_dev,
                        void* stream);

/* counter[0] += v on the device (a one-thread kernel: capturable, unlike a
 * host write). */
int sil_unet_counter_add(int32_t* counter, int32_t v, void* stream);

#define SIL_UNET_W_CONV3 1 /* w [cout][3][3][cin]; wt [cin][3][3][cout] flipped (sil_unet_flip3x3) */
#define SIL_UNET_W_UP2 2   /* w [2][2][cout][cin]; wt [cin][2][2][cout] (sil_unet_up_t) */

/* One weight tensor to prepare for a forward and backward pass: wb = bf16(w)
 * in w's layout, and (wt non-NULL) the bf16 transposed form the input
 * gradient uses. */
typedef struct sil_unet_weight_prep {
  const float* w;
  void* wb;
  void* wt;
  int32_t kind;
  int32_t cout, cin;
} sil_unet_weight_prep;

/* bf16 weight copies and transposed forms for `count` tensors in one launch
 * per 64 tensors (round to nearest even, as sil_unet_to_bf16). */
int sil_unet_prep_weights(const sil_unet_weight_prep* t, int32_t count, void* stream);

/* One batch-norm layer's per-channel vectors (fp32 [C]; C <= 256). */
typedef struct sil_unet_bn_layer {
  int32_t C;
  const float* mr;      /* [2][C] batch (mean, rstd), from sil_unet_bn_relu */
  float* running_mean;
  float* running_var;
  const float* gamma;
  const float* beta;
  float* scale;         /* inference: gamma / sqrt(running_var + eps) */
  float* shift;         /* inference: beta - running_mean * scale */
} sil_unet_bn_layer;

/* Running statistics as an exponential moving average of the batch
 * statistics: running_mean = (1 - momentum) running_mean + momentum mean,
 * running_var likewise with the biased batch variance 1/rstd^2 - eps, for
 * `count` layers (mr, running_mean, running_var used). */
int sil_unet_bn_ema(const sil_unet_bn_layer* l, int32_t count, float momentum, float eps,
                    void* stream);

/* Inference scale and shift from the running statistics for `count` layers
 * (running_mean, running_var, gamma, beta, scale, shift used). */
int sil_unet_bn_fold(const sil_unet_bn_layer* l, int32_t count, float eps, void* stream);

/* fp32 -> bf16 (round to nearest even). */
int sil_unet_to_bf16(const float* x, void* y, int64_t n, void* stream);

/* x[i] = v for i < n (fp32 fill, e.g. to zero accumulators). */
int sil_unet_fill_f32(float* x, int64_t n, float v, void* stream);

#ifdef __cplusplus
}
#endif
#endif
