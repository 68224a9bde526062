/* fmbym_mask.h - C ABI of the learned mask network and its training step.
 *
 * Section III-E: a network h_alpha maps the scans to masks in (0, 1)^(n x n)
 * (Eq. 10); the search runs on the masked scans (Eq. 11-12, the m_f / m_g
 * arguments of fmbym_search) and the network is trained end to end on the
 * pose error (Eq. 13) with Adam.  The network follows the pattern of
 * Table II (a U-Net of 3x3 convolutions with BatchNorm and ReLU, max-pooling
 * down, bilinear upsampling and skip concatenation up, a sigmoid head), sized
 * by `levels`, `base_channels` and `channels`:
 *   level l (0 <= l < levels) works at side n >> l with base_channels << l
 *   channels; encoder level l: [2x2 max-pool if l > 0], conv a, conv b;
 *   decoder level l (levels-2 >= l >= 0): concat[up2(deeper), skip l], conv a,
 *   conv b; head: 3x3 conv (with bias) to `channels` outputs, sigmoid.
 * Every conv is 3x3, padding 1, no bias, followed by BatchNorm and ReLU.
 * BatchNorm normalises with the batch statistics (biased variance) when
 * training and with the running statistics otherwise; the running statistics
 * move by `bn_momentum` towards the batch mean and the unbiased batch variance.
 * up2 is bilinear x2 with half-pixel centres: output o samples the source at
 * max(0, (o + 1/2)/2 - 1/2), the upper neighbour clamped at the edge.
 * channels = 1 (or 0): one call processes `images` single scans, and the
 * scans f and g of a pair both go through the same network (x and mask are
 * [images][n][n]).  channels = 2: Table II's dual-input network (6 levels,
 * 8 -> 256 channels, about 1.97 M weights) sees both scans of a pair as two
 * input channels and returns both masks; x and mask are [2][images][n][n],
 * plane 0 holding f (m_f) and plane 1 g (m_g) of every pair, which is the
 * layout of the f batch followed by the g batch.
 *
 * Arithmetic: convolutions on the matrix cores in BF16 with FP32
 * accumulation; activations are stored in BF16 (NHWC); BatchNorm statistics,
 * the head, the sigmoid, all gradients outside the convolution operands and the
 * optimiser run in FP32.
 *
 * Flat FP32 parameter vector (params, d_params, Adam moments): for each
 * convolution in the order enc0a, enc0b, enc1a, enc1b, ..., dec(levels-2)a,
 * dec(levels-2)b, ..., dec0a, dec0b: weight [c_out][c_in][3][3], gamma [c_out],
 * beta [c_out]; then the head weight [channels][base_channels][3][3] and its
 * bias [channels].
 * BatchNorm running statistics: the means of every BN channel in the same
 * conv order, then their variances.
 *
 * Memory and errors as in fmbym.h: device pointers owned by the caller,
 * asynchronous on `stream`, validation before anything is enqueued, negative
 * FMBYM_E* codes.  Only fmbym_mask_pack reads params; call it after every
 * change of params (fmbym_adam does not re-pack).
 */
#ifndef FMBYM_MASK_H
#define FMBYM_MASK_H

#include "fmbym.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmbym_mask_desc_s {
    int32_t levels;          /* 1..6                                                      */
    int32_t base_channels;   /* 8                                                         */
    float bn_eps;            /* BatchNorm epsilon, > 0 (1e-5)                             */
    float bn_momentum;       /* running-statistics momentum in [0, 1] (0.1)               */
    float* params;           /* FP32 [fmbym_mask_param_count]                             */
    void* packed;            /* fmbym_mask_packed_bytes: BF16 weights as the kernels read  */
    float* bn_running;       /* FP32 [2 * fmbym_mask_bn_channels]                         */
    int32_t channels;        /* input scans and output masks per sample: 1 (0 reads as 1)
                                or 2 (the dual-input network)                               */
} fmbym_mask_desc;

#define FMBYM_LOSS_L1 1      /* Eq. 13: sum of |error| over (theta, t_x, t_y), batch mean  */
#define FMBYM_LOSS_L2 2      /* squared errors instead                                     */

/* Sizes of the buffers a descriptor points to; 0 if levels/base_channels are unsupported. */
FMBYM_API size_t fmbym_mask_param_count(const fmbym_mask_desc* net);
FMBYM_API size_t fmbym_mask_packed_bytes(const fmbym_mask_desc* net);
FMBYM_API size_t fmbym_mask_bn_channels(const fmbym_mask_desc* net);

/* Convert params to the BF16 operand layouts in `packed` (forward and data-gradient). */
FMBYM_API int fmbym_mask_pack(const fmbym_mask_desc* net, void* stream);

/* Bytes of the activation buffer of fmbym_mask_fwd / fmbym_mask_bwd for
 * `images` samples of side n (n = 128, 256 or 512 and n >> (levels-1) >= 16,
 * so 6 levels need n = 512); 0 on bad input. */
FMBYM_API size_t fmbym_mask_activation_bytes(const fmbym_mask_desc* net, int32_t images, int32_t n);

/* Forward pass: x [channels][images][n][n] scans -> mask [channels][images][n][n] in (0, 1).
 * training != 0 uses batch statistics, updates bn_running and saves in act
 * every activation fmbym_mask_bwd reads (it is required before the backward);
 * training == 0 uses bn_running and uses act as scratch only (the layer
 * outputs, not the saved state of a training forward). */
FMBYM_API int fmbym_mask_fwd(const fmbym_mask_desc* net, int32_t images, int32_t n, const float* x,
                             float* mask, void* act, size_t act_bytes, int training, void* stream);

/* Bytes of scratch workspace for fmbym_mask_bwd; 0 on bad input. */
FMBYM_API size_t fmbym_mask_workspace_bytes(const fmbym_mask_desc* net, int32_t images, int32_t n);

/* Backward pass of a training forward: given d_mask = dL/dmask [images][n][n]
 * and the forward's act, writes dL/dparams (FP32, flat layout, overwritten)
 * and, unless d_x is NULL, dL/dx [channels][images][n][n] (FP32, overwritten): the
 * gradient of the loss with respect to the network's input scans (the
 * straight-through derivative of their BF16 rounding), for a caller that
 * trains what produces the scans or checks the network's sensitivity.
 * The weight gradients run on a second stream the library keeps per device,
 * forked from and joined back into `stream` with events, so the call's work
 * is complete when `stream`'s is (a graph capture of `stream` takes both);
 * calls from several host threads enqueue one at a time. */
FMBYM_API int fmbym_mask_bwd(const fmbym_mask_desc* net, int32_t images, int32_t n,
                             const float* d_mask, const void* act, size_t act_bytes, float* d_params,
                             float* d_x, void* workspace, size_t workspace_bytes, void* stream);

/* Adam (bias-corrected, step >= 1) over `count` FP32 parameters in place. */
FMBYM_API int fmbym_adam(float* params, const float* grad, float* m, float* v, int64_t count,
                         int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/* Pose loss of Eq. 13 over a batch: loss[0] = mean_b sum_j e(pose[b][j] - target[b][j])
 * with e = |.| (FMBYM_LOSS_L1) or (.)^2 (FMBYM_LOSS_L2); d_pose [batch][3] = dloss/dpose. */
FMBYM_API int fmbym_pose_loss(int32_t batch, const float* pose, const float* target, int32_t kind,
                              float* loss, float* d_pose, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FMBYM_MASK_H */
