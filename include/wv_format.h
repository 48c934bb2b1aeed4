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

/* Record runs of the visible tiles of one plane of one frame (Section 3.4: a
 * run of blocks is read with two block-end pointers).  For every tile with
 * tile_mask[t] != 0, the blocks that level_count[t] keeps (NULL = all levels;
 * Section 3.7) are a prefix of the tile's level-wise block order, so their
 * records form one range [first record of the tile, end of its last kept
 * block); ranges of consecutive visible tiles that touch are merged.  Host
 * only, no device work.
 *  block_end : HOST [n_tiles * nb], the plane's block ends; ends beyond
 *              n_records count as n_records.
 *  run_begin, run_end : HOST int64 [n_tiles] (room for one run per tile);
 *              runs in ascending order, run_begin < run_end, empty ranges
 *              omitted.
 *  n_runs, n_in_runs : HOST outputs: runs written, records they hold.
 * Errors: WV_EINVAL (geometry, plane, NULL, a level count above levels, block
 * ends of a visible tile that decrease). */
wv_status wv_sparse_visible_runs(const wv_desc* desc, int32_t plane, const uint32_t* block_end,
                                 int64_t n_records, const uint8_t* level_count,
                                 const uint8_t* tile_mask, int64_t* run_begin, int64_t* run_end,
                                 int32_t* n_runs, int64_t* n_in_runs);

/* Asynchronous prefetch of a sparse store kept in host memory (Section 3.5,
 * Fig. 4): the frames of the next inter-frame set are staged -- the visible
 * tiles' record runs gathered and uploaded on a copy stream of the prefetcher
 * -- while the GPU rebuilds and decodes the previous set.  Two staging slots
 * (pinned host + device) alternate; each set is staged once and rebuilt
 * once, in order.  The prefetcher belongs to one context (its geometry and
 * device); calls on one prefetcher must not overlap. */
typedef struct wv_prefetch wv_prefetch;

/* max_frames: frames per staged set (1 .. 16); slot_bytes: capacity of each
 * of the two staging slots (host and device), 1 KiB .. 2^40.
 * Errors: WV_EINVAL, WV_ENOMEM, WV_EDEVICE. */
wv_status wv_prefetch_create(wv_ctx* ctx, int32_t max_frames, int64_t slot_bytes,
                             wv_prefetch** out);
/* Waits for the prefetcher's copies and rebuilds, then frees it (NULL is a
 * no-op).  Destroy a prefetcher before its context. */
wv_status wv_prefetch_destroy(wv_prefetch* pf);

/* Stage n_frames frames for one viewport.
 *  frames : HOST [n_frames * nplanes] (frame-major) sparse planes whose
 *           block_end, values and index point to HOST memory, the store.
 *  level_count, tile_mask : HOST [n_tiles], as for wv_decode_viewport.
 *  direct : 0 = the CPU gathers the runs into the slot's pinned staging
 *           buffer and one copy uploads the slot; 1 = one copy per run
 *           straight from the store (which must then be pinned, e.g. from
 *           hipHostMalloc) and one for the staged block-end tables.
 *  bytes  : HOST output (may be NULL), bytes uploaded for the set.
 * Per frame and plane the slot holds the visible tiles' block ends rebased
 * to the staged records (uint32 [n_visible * nb]), then their indices and
 * codes.  The call checks the set and computes its record runs, then returns:
 * the prefetcher's own thread (the paper's prepare thread) gathers the runs
 * and enqueues the copies on the prefetcher's copy stream, after the slot's
 * previous rebuild.  The store (the arrays frames point to) must stay valid
 * and unchanged until the set has been rebuilt (or the prefetcher
 * destroyed); tile_mask and level_count
 * are read during the call only.  At most two sets may be staged and not yet
 * rebuilt.
 * Errors: WV_EINVAL (arguments, a level count above levels, a third staged
 * set, n_frames above max_frames, more bytes than slot_bytes; nothing is
 * enqueued then), WV_EDEVICE. */
wv_status wv_prefetch_stage(wv_prefetch* pf, const wv_sparse_plane* frames, int32_t n_frames,
                            const uint8_t* level_count, const uint8_t* tile_mask, int32_t direct,
                            int64_t* bytes);

/* Rebuild the oldest staged set on `stream` (which first waits for its
 * upload; the call itself waits until the prepare thread has enqueued that
 * upload, and reports its errors): frame f, plane p is written into
 * dense[f * nplanes + p] exactly
 * as wv_sparse_rebuild writes it (visible tiles, kept levels; device,
 * 16-byte aligned, [n_tiles][P][P] int16 for 5/3, float32 for 9/7).  The
 * slot is free for the next stage once this work has run.
 *  dense : HOST array [n_frames * nplanes] of device pointers.
 * Errors: WV_EINVAL (nothing staged, NULL or misaligned planes), WV_EDEVICE. */
wv_status wv_prefetch_rebuild(wv_prefetch* pf, void* const* dense, hipStream_t stream);

/* The file of a sequence of frames in the format (Section 3.4): a header
 * (magic "WV360FMT", version 1, the geometry, frame count), then a metadata
 * table with one entry per frame and plane (file offset of its packages,
 * record count, the four Eq. 4 bounds), then per frame and plane a block-end
 * package (uint32 [n_tiles * nb]) followed by its coefficient package (the
 * uint16 indices, then the uint8 codes), each package 16-byte aligned in the
 * file.  Block ends are the in-memory ones (cumulative over the plane's
 * records).  Little-endian, as every target of this library is.
 *  frames : HOST [n_frames * nplanes] (frame-major) planes with HOST arrays.
 * Errors: WV_EINVAL (geometry, NULL, n_frames < 1), WV_EDEVICE (the file
 * cannot be written; the message names the path). */
wv_status wv_store_write(const char* path, const wv_desc* desc, int32_t n_frames,
                         const wv_sparse_plane* frames);

/* A file read whole into host memory: the store the prefetcher stages from
 * (the paper's RAM buffers; its block ends preloaded with the rest). */
typedef struct wv_store wv_store;
/* pinned != 0: page-locked memory (hipHostMalloc), which a copy per run
 * (wv_prefetch_stage with direct = 1) needs; 0: ordinary memory.
 * Errors: WV_EINVAL (NULL, not a file of this format, truncated or
 * inconsistent), WV_ENOMEM, WV_EDEVICE (read error). */
wv_status wv_store_open(const char* path, int32_t pinned, wv_store** out);
wv_status wv_store_close(wv_store* store);
/* The file's geometry and frame count. */
wv_status wv_store_info(const wv_store* store, wv_desc* desc, int32_t* n_frames);
/* The planes of frame f, pointing into the store (valid until it is closed).
 *  planes : HOST [nplanes] outputs. */
wv_status wv_store_frame(const wv_store* store, int32_t frame, wv_sparse_plane* planes);

#ifdef __cplusplus
}
#endif
#endif /* WV_FORMAT_H */
