/*
 * lddmm_cnn.h -- kernels of the warm-start network (MI355X, gfx950).
 *
 * The paper starts every registration from v = 0 (Methods, Registration:
 * gradient descent on the velocity).  This library adds a learned initial
 * velocity: a small 3-D convolutional encoder-decoder maps the mask pair
 * (M0, M1) to v at a quarter of the resolution; the paper's descent then
 * refines it and stays the judge of its error.  These are the calls that train
 * and run that network on the GPU.
 *
 * Conventions shared by every call:
 *  - All pointers are DEVICE pointers owned by the caller; nothing is
 *    allocated or freed here.  `stream` is a hipStream_t passed as void*;
 *    every call is asynchronous on it and reports launch errors only.
 *  - Tensors are channels-last: element (b, z, y, x, c) of a tensor with
 *    geometry {n, d, h, w, c} sits at (((b d + z) h + y) w + x) c + c.
 *  - bf16 values are IEEE binary32 truncated to the top 16 bits, passed as
 *    uint16_t; rounding to bf16 is to nearest, ties to even.  Sums accumulate
 *    in FP32 on the matrix cores; energies and losses in FP64.
 *  - A 3x3x3 convolution with stride s in {1, 2} and zero padding 1 maps
 *    extent n to (n - 1)/s + 1.  Weights are w[co][kz][ky][kx][ci] (bf16),
 *    biases FP32.
 *  - Status: LDDMM_OK, or LDDMM_EINVAL for a null pointer, a non-positive
 *    size, a stride other than 1 or 2, an element count of 2^31 or more, or a
 *    workspace that is too small; LDDMM_EHIP for a launch failure.
 */
#ifndef LDDMM_CNN_H
#define LDDMM_CNN_H

#include <stddef.h>
#include <stdint.h>

#include "lddmm.h"   /* status codes */

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n, d, h, w, c;          /* samples, extents (z, y, x), channels */
} lddmm_cnn_shape;

#define LDDMM_CNN_BF16 0
#define LDDMM_CNN_F32  1

/* y = act(conv(x, w) + bias): x {n,d,h,w,cin} bf16, w [cout][27 cin] bf16, bias
 * [cout] FP32 (may be NULL: zero), relu 0/1, y {n, d', h', w', cout} of dtype
 * y_dtype (LDDMM_CNN_BF16 or LDDMM_CNN_F32). */
int lddmm_conv3d_forward(const uint16_t *x, lddmm_cnn_shape xs, const uint16_t *w,
                         const float *bias, int32_t cout, int32_t stride, int32_t relu, void *y,
                         int32_t y_dtype, void *stream);

/* Input gradient of lddmm_conv3d_forward for the output gradient dy (bf16, the
 * output geometry): dx = conv^T(dy), then optionally dx *= 1[mask > 0] (mask:
 * bf16 tensor of x's geometry, typically the forward input when it is a ReLU
 * output) and dx += add[vox * add_stride + add_off + c] (add: bf16, x's voxels
 * with add_stride channels).  wt is the weight transposed to [cin][27 cout]
 * (lddmm_cnn_transpose_weight).  dx {x's geometry} of dtype dx_dtype. */
int lddmm_conv3d_backward_data(const uint16_t *dy, lddmm_cnn_shape xs, int32_t cout,
                               int32_t stride, const uint16_t *wt, const uint16_t *mask,
                               const uint16_t *add, int32_t add_stride, int32_t add_off, void *dx,
                               int32_t dx_dtype, void *stream);

/* Bytes of workspace lddmm_conv3d_backward_weight needs for this geometry. */
size_t lddmm_conv3d_wgrad_workspace(lddmm_cnn_shape xs, int32_t cout, int32_t stride);

/* Weight and bias gradients: dw[co][k][ci] = sum over samples and output voxels
 * of dy[o][co] x[s o + k - 1][ci] (FP32, overwritten); db[co] = sum of dy[o][co]
 * (FP32, overwritten; may be NULL).  The sum over voxels is split across
 * blocks and reduced in a fixed order, so results are deterministic. */
int lddmm_conv3d_backward_weight(const uint16_t *dy, const uint16_t *x, lddmm_cnn_shape xs,
                                 int32_t cout, int32_t stride, float *dw, float *db,
                                 void *workspace, size_t workspace_bytes, void *stream);

/* wt[ci][k][co] = w[co][k][ci] (bf16). */
int lddmm_cnn_transpose_weight(const uint16_t *w, int32_t cout, int32_t cin, uint16_t *wt,
                               void *stream);

/* FP32 -> bf16 (round to nearest even) of `count` values. */
int lddmm_cnn_to_bf16(const float *src, int64_t count, uint16_t *dst, void *stream);

/* Nearest 2x upsampling of `coarse` {n,d,h,w,cc} concatenated with `skip`
 * {n,2d,2h,2w,cs}: out {n,2d,2h,2w,cc+cs} (bf16). */
int lddmm_cnn_upcat(const uint16_t *coarse, lddmm_cnn_shape cs, const uint16_t *skip,
                    int32_t skip_c, uint16_t *out, void *stream);

/* Gradient of lddmm_cnn_upcat in `coarse`: d_coarse[p][c] = sum over the 8
 * children q of p of dcat[q][c] for c < cs.c (bf16 in and out); dcat has
 * cs.c + skip_c channels.  The skip part is a channel slice of dcat. */
int lddmm_cnn_upcat_backward(const uint16_t *dcat, lddmm_cnn_shape cs, int32_t skip_c,
                             uint16_t *d_coarse, void *stream);

/* Mean squared error over `count` FP32 values: *loss = mean (out - target)^2
 * (device FP64), dout = bf16(2 (out - target) / count). */
int lddmm_cnn_mse(const float *out, const float *target, int64_t count, uint16_t *dout,
                  double *loss, void *workspace, size_t workspace_bytes, void *stream);
size_t lddmm_cnn_mse_workspace(int64_t count);

/* One Adam step (Kingma and Ba) over `count` FP32 parameters p with gradient g
 * and moments m, v (updated in place); step >= 1 is the step count used for
 * the bias correction.  p_bf16 (may be NULL) receives bf16(p). */
int lddmm_cnn_adam(float *p, const float *g, float *m, float *v, int64_t count, int32_t step,
                   float lr, float beta1, float beta2, float eps, uint16_t *p_bf16, void *stream);

/* Network input of one registration: x[vox][0] = bf16(M0), x[vox][1] = bf16(M1)
 * over `count` voxels. */
int lddmm_cnn_pack_masks(const float *M0, const float *M1, int64_t count, uint16_t *x,
                         void *stream);

/* Training label of one registration: v [T][3][d][h][w] (FP32, d, h, w
 * multiples of 4) averaged over 4x4x4 blocks, times `scale`, written
 * channels-last as label[d/4][h/4][w/4][3T] with channel 3j + component. */
int lddmm_cnn_pool_velocity(const float *v, int32_t T, int32_t d, int32_t h, int32_t w,
                            float scale, float *label, void *stream);

/* Initial velocity from a network output out[d][h][w][3T] (FP32) on a grid 4x
 * coarser than the computational grid {4d, 4h, 4w}: times `scale`, then two
 * cell-centred trilinear 2x upsamplings (the pyramid transfer of
 * lddmm_register), into v [T][3][4d][4h][4w].  `scratch` holds
 * 3T (2d)(2h)(2w) + 3T d h w floats. */
int lddmm_cnn_expand_velocity(const float *out, int32_t T, int32_t d, int32_t h, int32_t w,
                              float scale, float *v, float *scratch, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LDDMM_CNN_H */
