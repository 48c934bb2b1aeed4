/* wv_format.h -- the paper's sparse storage format and its GPU rebuild (libwv).
 *
 * Sections 3.3, 3.4 and 3.6: a frame's wavelet coefficients are thresholded
 * (Eq. 2 with the level-weighted threshold of Eq. 3 and the pole factor H(y)
 * of Section 3.6), quantised to 8 bits between a minimum and a maximum (Eq. 4;
 * one pair for the approximation band and one for the detail bands), and
 * stored sparsely as (code, position) records grouped in 32 x 32 blocks with
 * one block-end pointer per block.  Section 3.5 rebuilds the wavelet image on
 * the GPU from the records of the viewport before the inverse transform.
 *
 * Layout of one plane of one frame (tile-major like the coefficient planes of
 * wv.h; P = the plane's tile edge, B = min(32, P), nb = (P / B)^2 blocks per
 * tile):
 *  - blocks of a tile in level-wise order from the lowest frequency: a block's
 *    level is the level of the detail region its origin lies in (the block
 *    holding the approximation comes first), row-major within a level, so
 *    the blocks of the finest levels are a tile's trailing records;
 *  - records: values[r] (uint8 Eq. 4 code) and index[r] (uint16, y * B + x
 *    inside the block), ascending index within a block;
 *  - block_end[t * nb + j]: exclusive end of block j of tile t in the record
 *    arrays (cumulative over the plane);
 *  - bounds = {approximation min, max, detail min, max} (float32).
 * A record decodes to c = min + code * float32((max - min) / 255) in float32
 * (product and sum each rounded once); positions without a record are zero.
 *
 * Readings of the paper (it leaves them open): coefficients compare with T on
 * the 0..1 colour scale (|c| / 255 > T keeps c); in Eq. 3 l = k - 1 for detail
 * level k (1 = finest) and l_max = levels, so the finest details get
 * T = alpha + H; y is the centre row of the samples a coefficient covers,
 * within its eye (frames are top-bottom stereo, S_y = eye height); the
 * approximation band is never thresholded.
 */
#ifndef WV_FORMAT_H
#define WV_FORMAT_H

#include "wv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One plane of one frame in the sparse format, on the device. */
typedef struct {
  const uint32_t* block_end;  /* [n_tiles * nb] */
  const uint8_t* values;      /* [n_records] */
  const uint16_t* index;      /* [n_records] */
  int64_t n_records;
  float bounds[4];            /* approximation min, max; detail min, max */
} wv_sparse_plane;

/* Blocks per tile of plane p of a geometry (0 if p is not a plane of it). */
int32_t wv_sparse_blocks_per_tile(const wv_desc* desc, int32_t plane);

/* Encode one plane of one frame (host, offline; Eq. 2-4).
 *  coef      : HOST float32 [n_tiles][P][P], wavelet coefficients of plane p on
 *              the 0..255 scale, Mallat order per tile.
 *  alpha     : Eq. 3's constant (0 keeps every non-zero coefficient).
 *  poles     : nonzero adds H(y) = 1 - sin(pi y / S_y) to every threshold.
 *  block_end : HOST [n_tiles * nb]; values, index: HOST, room for
 *              n_tiles * P * P records (every coefficient kept).
 *  n_records, bounds : HOST outputs.
 * Errors: WV_EINVAL (geometry, plane, NULL, alpha < 0 or not finite). */
wv_status wv_sparse_encode_plane(const wv_desc* desc, int32_t plane, const float* coef, double alpha,
                                 int32_t poles, uint32_t* block_end, uint8_t* values, uint16_t* index,
                                 int64_t* n_records, float* bounds);

/* Rebuild the dense coefficient planes of the visible tiles (Section 3.5):
 * for every tile with tile_mask[t] != 0, the blocks of the levels that
 * level_count[t] keeps (Section 3.7; NULL = all) are written in full into
 * dense[p] (device, [n_tiles][P][P], int16 = the nearest integer of the
 * decoded value for a 5/3 context, float32 for 9/7); other blocks and tiles
 * are not written.  A decode of the same tiles with the same level counts
 * (wv_decode_viewport with an intra frame of qstep 1, or the bands of
 * wv_decode_set) then runs on dense.  planes: HOST array [nplanes].  Records
 * whose index lies outside their block, and block ends beyond n_records, are
 * ignored.  Errors: WV_EINVAL, WV_EDEVICE. */
wv_status wv_sparse_rebuild(wv_ctx* ctx, const wv_sparse_plane* planes, const uint8_t* level_count,
                            const uint8_t* tile_mask, void* const* dense, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* WV_FORMAT_H */
