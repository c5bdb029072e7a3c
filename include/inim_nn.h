/*
 * inim_nn.h -- C ABI of the layers of the learned surrogate: a convolutional
 * network that maps a density raster to the displacement of the whole
 * iterated regularisation (the composite map of Sec. 4.3 minus the identity),
 * trained on fields that the method itself computes (inim_regularize_probes).
 * The surrogate is not part of the paper; the paper's method stays its
 * fallback and its reference.
 *
 * Conventions
 *   - Tensors are device memory owned by the caller, NHWC: [images][h][w][c]
 *     with channels contiguous.  BF16 values are bfloat16 bit patterns
 *     (inim_bf16); FP32 values are float.
 *   - Convolution weights are [cout][ks*ks][cin] (taps in row-major (ky, kx)
 *     order), stride 1, zero padding ks/2 ("same" size); ks is 1 or 3.
 *     Channel counts of convolutions are positive multiples of 8.
 *   - Products are of BF16 operands, exact in FP32; sums are FP32 (on the
 *     matrix cores) in an order that depends only on the shapes, so results
 *     are deterministic.
 *   - Work is enqueued on `stream`; nothing is allocated or synchronised.
 *   - Return INIM_OK, INIM_EINVAL (bad shape or NULL), INIM_ERANGE (2^31 or
 *     more pixels), INIM_EWORKSPACE or INIM_EHIP; the text of the last error
 *     of this thread is inim_nn_last_error().
 */
#ifndef INIM_NN_H
#define INIM_NN_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef uint16_t inim_bf16;

const char* inim_nn_last_error(void);

/* Device work buffer for the three calls below on a layer of this shape:
 * FP32 partial sums of the K range split into slices when the output alone
 * has too few 128 x 128 tiles to fill the GPU.  The slices are added in a
 * fixed order, so results do not depend on timing.  When h and w are powers
 * of two and w is a multiple of 8, it also holds channel-major copies of the
 * weight gradient's operands x and dy (2 (cin + cout) bytes per pixel).  The
 * buffer must be 256-byte aligned (as hipMalloc returns it). */
int inim_conv_workspace(int32_t imgs, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t ks, size_t* bytes);

/* y[p][co] = act(bias[co] + sum over taps t and cin of x[p + off_t][ci] w[co][t][ci]);
 * act = max(., 0) when relu != 0.  bias may be NULL.  Writes y16 (BF16) and/or
 * y32 (FP32) when not NULL.  work may be NULL (no split of the K range). */
int inim_conv_forward(const inim_bf16* x, int32_t imgs, int32_t h, int32_t w, int32_t cin, const inim_bf16* weight,
                      const float* bias, int32_t cout, int32_t ks, int32_t relu, inim_bf16* y16, float* y32, void* work,
                      size_t work_bytes, hipStream_t stream);

/* Gradient of the input: dx[q][ci] = sum over t and co of dy[q - off_t][co] w[co][t][ci],
 * with weight_t = inim_weight_transpose(weight) = [cin][ks*ks][cout].  FP32 dx.
 * work may be NULL (no split of the K range). */
int inim_conv_backward_data(const inim_bf16* dy, int32_t imgs, int32_t h, int32_t w, int32_t cin,
                            const inim_bf16* weight_t, int32_t cout, int32_t ks, float* dx, void* work,
                            size_t work_bytes, hipStream_t stream);

/* Gradient of the weights and bias: dweight[co][t][ci] = sum over pixels p of
 * dy[p][co] x[p + off_t][ci]; dbias[co] = sum over p of dy[p][co] (dbias may be
 * NULL).  FP32; work of inim_conv_workspace bytes (required) holds the partial
 * sums over slices of the pixels. */
int inim_conv_backward_weight(const inim_bf16* dy, const inim_bf16* x, int32_t imgs, int32_t h, int32_t w, int32_t cin,
                              int32_t cout, int32_t ks, float* dweight, float* dbias, void* work, size_t work_bytes,
                              hipStream_t stream);

/* weight_t[ci][t][co] = weight[co][t][ci] */
int inim_weight_transpose(const inim_bf16* weight, int32_t cout, int32_t ks, int32_t cin, inim_bf16* weight_t,
                          hipStream_t stream);

/* b[i] = bfloat16(a[i]), round to nearest even. */
int inim_f32_to_bf16(const float* a, int64_t n, inim_bf16* b, hipStream_t stream);

/* 2 x 2 average pooling of an h x w image (h, w even) into (h/2) x (w/2). */
int inim_pool2(const inim_bf16* x, int32_t imgs, int32_t h, int32_t w, int32_t c, inim_bf16* y, hipStream_t stream);
/* Its gradient: dx (h x w) = dy (h/2 x w/2) / 4 per covered pixel; added to dx when accumulate != 0. */
int inim_pool2_backward(const float* dy, int32_t imgs, int32_t h, int32_t w, int32_t c, float* dx, int32_t accumulate,
                        hipStream_t stream);

/* Nearest 2x upsampling of an h x w image into channels [c0, c0 + c) of the
 * ct-channel 2h x 2w tensor y (the first half of a channel concatenation). */
int inim_upsample2_into(const inim_bf16* x, int32_t imgs, int32_t h, int32_t w, int32_t c, inim_bf16* y, int32_t ct,
                        int32_t c0, hipStream_t stream);
/* y[p][c0 + c'] = x[p][c'] for c' < c (the second half of a concatenation). */
int inim_copy_channels_into(const inim_bf16* x, int64_t pixels, int32_t c, inim_bf16* y, int32_t ct, int32_t c0,
                            hipStream_t stream);
/* The decoder's concatenation in one pass: y (imgs x 2h x 2w, ca + cb
 * channels) = [inim_upsample2_into(a) | b], a imgs x h x w x ca, b
 * imgs x 2h x 2w x cb; the same values as the two calls above. */
int inim_concat_up2(const inim_bf16* a, int32_t imgs, int32_t h, int32_t w, int32_t ca, const inim_bf16* b,
                    int32_t cb, inim_bf16* y, hipStream_t stream);
/* Gradient of inim_upsample2_into for c0 = 0: da (h x w, ca channels) = sum of
 * the 2 x 2 block of dy (2h x 2w, ct channels), channels [0, ca). */
int inim_upsample2_backward(const float* dy, int32_t imgs, int32_t h, int32_t w, int32_t ct, int32_t ca, float* da,
                            hipStream_t stream);
/* out[p][c'] (+)= dy[p][c0 + c'] for c' < c: the gradient of a copied half. */
int inim_take_channels(const float* dy, int64_t pixels, int32_t ct, int32_t c0, int32_t c, float* out,
                       int32_t accumulate, hipStream_t stream);

/* g16 = bfloat16(g * (act > 0)), act = the ReLU layer's output (NULL: no mask). */
int inim_relu_backward(const float* g, const inim_bf16* act, int64_t n, inim_bf16* g16, hipStream_t stream);

/* Mean-squared error of the first ct of cp predicted channels against target
 * [pixels][ct]: *loss (device) = sum of squared differences; grad (may be NULL)
 * = 2 (pred - target) / (pixels ct) as BF16, 0 in the other channels.  work:
 * at least 1 KiB of device memory. */
int inim_mse(const float* pred, int32_t cp, const float* target, int32_t ct, int64_t pixels, float* loss,
             inim_bf16* grad, void* work, size_t work_bytes, hipStream_t stream);

/* One Adam step (bias-corrected, step >= 1) on FP32 weights with FP32
 * moments m and v; also writes the BF16 copy weight16 when not NULL. */
int inim_adam(float* weight, const float* grad, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
              int32_t step, inim_bf16* weight16, hipStream_t stream);

/* The network's input from a density raster (inim_rasterize): channel 0 of
 * x [res][res][c] = bfloat16(density * scale), the other channels 0. */
int inim_nn_pack_density(const float* density, int32_t res, float scale, int32_t c, inim_bf16* x, hipStream_t stream);

/* inim_nn_pack_density for a stack of `count` rasters (1..64): density
 * [count][res][res], x [count][res][res][c], raster q scaled by scale[q]
 * (host array). */
int inim_nn_pack_density_many(const float* density, int32_t count, int32_t res, const float* scale, int32_t c,
                              inim_bf16* x, hipStream_t stream);

/* The network's input with the method's first step: for `count` rasters
 * (1..64), channel 0 of x [count][res][res][c] (c >= 3) = bfloat16(density *
 * scale[q]) as in inim_nn_pack_density_many, channels 1 and 2 = bfloat16(64
 * (field - texel centre)), the displacement of one iteration of the method
 * (field: float [count][res][res][2], inim_deform of that density), and the
 * other channels 0.  The integral images behind that field sum the whole
 * raster, which the convolutions' finite reach cannot. */
int inim_nn_pack_input_many(const float* density, const float* field, int32_t count, int32_t res, const float* scale,
                            int32_t c, inim_bf16* x, hipStream_t stream);

/* Training target from probes started at the texel centres and moved by the
 * whole iteration (inim_regularize_probes): out [res][res][2] = (probe -
 * texel centre) * 64, the displacement in units of 1/64 of the unit square
 * (the same scale at every raster size). */
int inim_nn_displacement(const float* probe, int32_t res, float* out, hipStream_t stream);

/* The deformation field of a network output y [res][res][c] (c >= 2):
 * field [res][res][2] = texel centre + (y[..][0..1] smoothed) / 64, for
 * inim_advect.  The smoothing is the separable normalised Gaussian of
 * standard deviation radius / 2 over |d| <= radius along x, then y (indices
 * clamped to the raster); radius 0..16, 0 = none.  work: device float
 * [res][res][2] for the intermediate pass. */
int inim_nn_field(const float* y, int32_t c, int32_t res, int32_t radius, float* field, float* work,
                  hipStream_t stream);

/* inim_nn_field for a stack of `count` outputs (1..65535): y
 * [count][res][res][c], field and work [count][res][res][2]; field q is the
 * one inim_nn_field gives for y[q]. */
int inim_nn_field_many(const float* y, int32_t count, int32_t c, int32_t res, int32_t radius, float* field, float* work,
                       hipStream_t stream);

/* Adds to *count (device) the number of lattice triangles (two per cell) of
 * the deformed texel lattice `field` with non-positive signed area (folds). */
int inim_nn_count_folds(const float* field, int32_t res, uint32_t* count, hipStream_t stream);

/* Adds to out[0], out[1] (device doubles) the sum of the per-bin sample
 * counts over bin x bin texel blocks and the sum of their squares. */
int inim_nn_bin_moments(const uint32_t* counts, int32_t res, int32_t bin, double* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* INIM_NN_H */
