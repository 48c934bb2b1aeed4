/* wv_cnn.h -- learned restoration of decoded viewports (libwv).
 *
 * A small convolutional network, not part of the paper, refines decoded
 * viewports of a coarsely quantised stream: four 3x3 convolutions
 * (3 -> 32 -> 32 -> 32 -> 3 channels), ReLU after the first three, and a
 * residual skip, y = x + z.  Convolutions run on bfloat16 MFMA with fp32
 * accumulation; parameters and optimiser state are fp32.  Trained on pairs of
 * (decoded, uncompressed) viewports that the codec itself produces, with the
 * plain decode kept as the fallback wherever a guard trips.
 *
 * Tensors are device buffers, NHWC with 4 channels for images (the 4th is
 * zero): x bfloat16 [n][h][w][4] with values in [0, 1], z and targets fp32
 * [n][h][w][4].  Parameters (fp32, wv_cnn_param_count() values): per layer,
 * W[out][3][3][in] then b[out], layers in order.
 *
 * All calls are stream-ordered on `stream`; a call returning WV_OK has
 * enqueued its work (calls that return host data synchronise first).
 * Errors: WV_EINVAL (bad argument or state), WV_ENOMEM, WV_EDEVICE.
 */
#ifndef WV_CNN_H
#define WV_CNN_H

#include "wv.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wv_cnn wv_cnn;

/* Number of fp32 parameters. */
int32_t wv_cnn_param_count(void);

/* Network with activation buffers for up to max_pixels = n * h * w pixels
 * (about 270 bytes of device memory per pixel).  Parameters start at zero:
 * set them before use. */
wv_status wv_cnn_create(wv_cnn** net, int64_t max_pixels);
wv_status wv_cnn_destroy(wv_cnn* net);

/* Copy parameters in (HOST fp32 array; resets the optimiser state) or out. */
wv_status wv_cnn_set_params(wv_cnn* net, const float* host_params, hipStream_t stream);
wv_status wv_cnn_get_params(wv_cnn* net, float* host_params, hipStream_t stream);

/* Forward pass of x; z = network output before the skip (fp32 NHWC4, may be
 * NULL: kept inside the network), written directly.  Keeps the activations
 * for wv_cnn_backward.  x is read in place, not copied: it (and z) must stay
 * unchanged until wv_cnn_loss_grad and wv_cnn_backward of this pass have
 * run. */
wv_status wv_cnn_forward(wv_cnn* net, const uint16_t* x, int32_t n, int32_t h, int32_t w, float* z,
                         hipStream_t stream);

/* The same forward pass for inference: z as for wv_cnn_forward (bit-identical
 * values), but the activations are not kept, so no wv_cnn_loss_grad or
 * wv_cnn_backward may follow it (they report WV_EINVAL).  x and z are only
 * read and written while the pass runs. */
wv_status wv_cnn_infer(wv_cnn* net, const uint16_t* x, int32_t n, int32_t h, int32_t w, float* z,
                       hipStream_t stream);

/* Mean squared error of x + z against t (fp32 NHWC4, 3 channels) for the
 * last forward pass, written to *loss (device float), and its gradient with
 * respect to z kept for wv_cnn_backward. */
wv_status wv_cnn_loss_grad(wv_cnn* net, const float* t, float* loss, hipStream_t stream);

/* Gradients of the loss with respect to every parameter (device fp32,
 * parameter layout; may be NULL to keep them internal for wv_cnn_adam). */
wv_status wv_cnn_backward(wv_cnn* net, float* grads, hipStream_t stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with the internal gradients;
 * step counts from 1. */
wv_status wv_cnn_adam(wv_cnn* net, float lr, int32_t step, hipStream_t stream);

/* forward + loss + backward + Adam. */
wv_status wv_cnn_train_step(wv_cnn* net, const uint16_t* x, const float* t, int32_t n, int32_t h,
                            int32_t w, float lr, int32_t step, float* loss, hipStream_t stream);

/* Square crops of tile-planar RGB viewports as network tensors.
 * images: device uint8 [n_images][tiles_y * tiles_x][3][tile][tile] (the
 * layout wv_decode_viewport writes for a viewport of tiles_y x tiles_x tiles
 * in row-major order); crops: HOST int32 [n_crops][3] = (image, y0, x0),
 * each inside its image; out: bfloat16 (as_float = 0) or fp32 NHWC4
 * [n_crops][size][size][4], values / 255.  At most 4096 crops.  Synchronous. */
wv_status wv_cnn_gather(wv_cnn* net, const uint8_t* images, int32_t tile, int32_t tiles_x,
                        int32_t tiles_y, int32_t n_images, const int32_t* crops, int32_t n_crops,
                        int32_t size, int32_t as_float, void* out, hipStream_t stream);

/* Restore one decoded viewport (tile-planar uint8 RGB as above) into `out`
 * (same layout).  Per tile, the network's output is kept only if every value
 * is finite and the mean absolute correction (on the 0..1 scale) is at most
 * `guard`; other tiles are the plain decode.  *fallback_tiles (HOST, may be
 * NULL) receives the number of tiles that fell back.  Synchronous. */
wv_status wv_cnn_restore(wv_cnn* net, const uint8_t* decoded, int32_t tile, int32_t tiles_x,
                         int32_t tiles_y, float guard, uint8_t* out, int32_t* fallback_tiles,
                         hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* WV_CNN_H */
