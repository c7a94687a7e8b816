/*
 * gs_nn.h - C ABI of the learned Gaussian initialiser and its plain
 * (cost-volume) counterpart in libgsmi.
 *
 * GEVO initialises new Gaussians from a depth image of the newest keyframe:
 * a photometric cost volume over the sliding window (Eq. 1, Sec. III-A1)
 * reduced to a depth per pixel (Sec. III-A2), from which Gaussians are
 * placed.  This library provides
 *   - the plain initialiser: the Eq. 1 cost volume at 1/4 resolution with 64
 *     depth hypotheses spaced evenly over 0.25-25 m, reduced by a
 *     winner-take-all argmin (the belief-propagation smoothing of Sec.
 *     III-A2 is not part of it), and
 *   - the building blocks of a small convolutional network that regresses
 *     per-pixel depth and Gaussian scale from one RGB image, trained on
 *     renders of the map: 3x3 convolutions as BF16 MFMA implicit GEMMs with
 *     FP32 accumulation, their data and weight gradients, 2x2 average
 *     pooling, nearest 2x upsampling, a 1x1 head and the depth loss.
 *
 * Conventions are those of gs.h (status codes, caller-owned memory,
 * asynchronous on the caller's stream, validation before launch).
 *
 * Activations are BF16 (raw uint16 storage) in NHWC layout described by
 * gs_act: element (n, y, x, c) is at
 *   data[((n * h + y) * w + x) * stride + offset + c],  0 <= c < c_count.
 * A view may select a channel slice of a wider tensor (stride > c, offset).
 * Convolution inputs and masks need c, stride and offset multiples of 8 and
 * 16-byte aligned data; padding channels up to the next multiple of 8 must
 * hold zeros.
 */
#ifndef GS_NN_H
#define GS_NN_H

#include "gs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_act {
  void* data;
  int32_t n, h, w;
  int32_t c;        /* channels of the view                     */
  int32_t stride;   /* elements between consecutive pixels       */
  int32_t offset;   /* first channel of the view within a pixel  */
} gs_act;

/* y = relu?(conv3x3(concat(x1, x2)) + bias), zero padding, stride 1.
 * x2 (optional) supplies channels after x1's (skip concatenation).
 * mask (optional, layout of the concatenated input): input entries whose mask
 * is <= 0 read as zero (fuses a ReLU backward into a backward-data call).
 * weights: BF16 [9][cout][cin] (tap = 3 dy + dx, dy, dx in 0..2).
 * bias: float32 [cout] or NULL.  Outputs: y (BF16 view with c = cout) and/or
 * y_f32 (float32, pixel stride y_f32_stride); either may be NULL, not both. */
int gs_nn_conv3x3(const gs_act* x1, const gs_act* x2, const gs_act* mask, const void* weights,
                  int32_t cout, const float* bias, int32_t relu, gs_act* y, float* y_f32,
                  int32_t y_f32_stride, gs_stream_t stream);

/* Weight and bias gradients of gs_nn_conv3x3, accumulated (+=) in float32:
 * dw [9][cout][cin] += sum_p dz[p][co] x[p + tap][ci], dbias[co] += sum_p dz[p][co],
 * with dz = dy masked by (mask > 0) when mask is given (mask is the layer's
 * ReLU output).  dbias may be NULL. */
int gs_nn_conv3x3_wgrad(const gs_act* x1, const gs_act* x2, const gs_act* dy, const gs_act* mask,
                        float* dw, float* dbias, gs_stream_t stream);

/* Backward-data weights: wt [9][cin][cout] = w [8 - tap][cout][cin], so that
 * gs_nn_conv3x3(dy, wt) gives the input gradient. */
int gs_nn_flip_weights(const void* weights, int32_t cout, int32_t cin, void* weights_t,
                       gs_stream_t stream);

/* 2x2 average pooling (h, w even): y (n, h/2, w/2, c). */
int gs_nn_avgpool2(const gs_act* x, gs_act* y, gs_stream_t stream);
/* dx = upsample(dy) / 4 (+ add, + dx if accumulate): dx has the full size. */
int gs_nn_avgpool2_bwd(const gs_act* dy, const gs_act* add, gs_act* dx, int32_t accumulate,
                       gs_stream_t stream);
/* Nearest 2x upsampling into y (n, 2h, 2w, c); y may be a channel slice. */
int gs_nn_upsample2(const gs_act* x, gs_act* y, gs_stream_t stream);
/* dx (n, h/2, w/2, c) = 2x2 block sums of dy (n, h, w, c). */
int gs_nn_upsample2_bwd(const gs_act* dy, gs_act* dx, gs_stream_t stream);

/* Planar float32 RGB [n][3][h][w] -> BF16 NHWC x (stride >= 3, channels
 * beyond 3 zeroed). */
int gs_nn_rgb_to_nhwc(const float* rgb, gs_act* x, gs_stream_t stream);
/* Round float32 to BF16 (nearest even), n elements. */
int gs_nn_f32_to_bf16(const float* src, void* dst, int64_t n, gs_stream_t stream);

/* 1x1 head: out [n][2][h][w] = b[k] + sum_c w[k][c] f[p][c] (float32 w [2][c]). */
int gs_nn_head(const gs_act* f, const float* w, const float* b, float* out, gs_stream_t stream);
/* Head backward: df (BF16, masked by f > 0, i.e. through the features'
 * ReLU), dw [2][c] and db [2] accumulated (+=). */
int gs_nn_head_bwd(const gs_act* f, const float* w, const float* dout, gs_act* df, float* dw,
                   float* db, gs_stream_t stream);

/* Depth supervision: pred [n][2][h][w] = (log depth, log scale), target depth
 * [n][h][w] (<= 0: no target).  L = mean over targets of
 * |pred0 - log d| + |pred1 - log(d / fx)|; dpred = dL/dpred (0 off target);
 * loss (optional, float64 [1]) overwritten with L.  ws: >= 8 bytes scratch. */
int gs_nn_depth_loss(const float* pred, const float* depth, int32_t n, int32_t h, int32_t w,
                     float fx, float* dpred, double* loss, void* ws, gs_stream_t stream);

/* Plain initialiser (Eq. 1 + winner-take-all).  keyframes: planar float32 RGB
 * [k][3][H][W] (device), cams: k cameras (host and device copies, as in
 * gs_views, all H x W); the reference is the last keyframe.  Intensity is
 * 0.299 R + 0.587 G + 0.114 B averaged over 4x4 blocks; low-resolution pixel
 * (i, j) sits at full-resolution (4 i + 2, 4 j + 2); source intensities are
 * sampled bilinearly on the low-resolution grid; views where the sample
 * falls outside the image (or behind the camera) are left out of the mean.
 * Outputs (device): cost [64][H/4][W/4] (optional; +inf where no view is
 * valid), depth [H/4][W/4] (0 where no hypothesis has a valid view).
 * ws: gs_cost_volume_workspace_size bytes. */
size_t gs_cost_volume_workspace_size(int32_t k, int32_t h, int32_t w);
int gs_cost_volume_wta(const float* keyframes, const gs_views* cams, float* cost, float* depth,
                       void* ws, size_t ws_bytes, gs_stream_t stream);

/* Depth from the cost volume by belief propagation (Sec. III-A2: a depth
 * image from the volume under a smoothness prior, Felzenszwalb and
 * Huttenlocher's loopy min-sum formulation).  cost: device float32
 * [64][h][w] as gs_cost_volume_wta writes it (+inf entries, hypotheses no
 * source view sees, cost `invalid_cost`).  On the 4-connected grid a pixel sends
 * each neighbour, for every label l' of the receiver,
 *   min over l of D(l) + (messages from its other three neighbours)(l)
 *                 + min(lam |l - l'|, trunc),
 * shifted to a zero minimum; messages start at 0 and are updated
 * synchronously `iters` times; a pixel's label is the first minimum of its
 * data cost plus its four incoming messages.  Outputs (device, optional
 * each): labels int32 [h][w], depth float32 [h][w] (the label's
 * hypothesis, 0.25 + 24.75 l / 63 m).  lam, trunc >= 0 and finite, iters
 * >= 0.  ws: gs_bp_workspace_size bytes (data costs and two message sets,
 * 9 x 64 floats per pixel). */
size_t gs_bp_workspace_size(int32_t h, int32_t w);
int gs_bp_labels(const float* cost, int32_t h, int32_t w, float lam, float trunc, int32_t iters,
                 float invalid_cost, int32_t* labels, float* depth, void* ws, size_t ws_bytes,
                 gs_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_NN_H */
