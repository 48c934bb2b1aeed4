/*
 * wv.h -- viewport-dependent wavelet decoding of 360-degree frames (C ABI).
 *
 * The operation (the paper's Section 3.1, 3.5-3.7): for each frame, only the
 * tiles inside the viewport are reconstructed.  Each visible tile gets a
 * multi-level 2D inverse wavelet transform (LeGall 5/3 integer lifting, or
 * CDF 9/7 in float32), with the finest levels' details treated as zero where
 * foveation drops them (Section 3.7); residual frames are then added onto the
 * previously decoded frame of the same tile, and YUV420 is converted to RGB.
 *
 * Conventions shared by every entry point:
 *  - A frame of width x height luma samples is cut into square tiles of
 *    `tile` samples (power of two); tiles are numbered row-major,
 *    t = ty * (width / tile) + tx.  Chroma planes (YUV420) are half size in
 *    both directions and use tiles of tile/2 that cover the same area.
 *  - Tile-major planes: plane p of a frame is an array
 *    [n_tiles][P][P] with P = tile (luma) or tile/2 (chroma); each tile's
 *    coefficients are in Mallat order (level k's region is the top-left
 *    P/2^(k-1) square; LL of the coarsest level in the top-left corner).
 *  - Transform conventions: whole-sample symmetric extension at tile edges;
 *    per inverse level, every row first, then every column; 5/3 uses floor
 *    division by arithmetic shift.  9/7 is the JPEG 2000 irreversible lifting
 *    (low band scaled by K, high band by 1/K on synthesis).
 *  - Device pointers are plain HIP device addresses (for instance from
 *    torch), at least 16-byte aligned.  The caller owns all buffers; the
 *    library never frees or keeps them beyond the stream-ordered work of the
 *    call.  Host pointers (masks, level counts, stamps) are read or written
 *    before the call returns.
 *  - Calls enqueue work on `stream` (NULL = the legacy default stream) and
 *    return; completion is stream-ordered.  No call throws; every call
 *    returns a wv_status.  On any error nothing has been enqueued and no
 *    caller-visible state (stamps included) has changed.
 *  - A context is used by one host thread at a time.
 */
#ifndef WV_H
#define WV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hipStream_t; /* HIP stream handle (same type as in HIP's headers) */

typedef enum {
  WV_OK = 0,
  WV_EINVAL = -1,        /* an argument is NULL, misaligned, out of range or inconsistent */
  WV_ESTALE = -2,        /* a residual frame's tile has no reconstruction of the previous frame */
  WV_ENOMEM = -3,        /* device or host allocation failed (set-up calls only) */
  WV_EDEVICE = -4,       /* a HIP call failed (message in wv_last_error) */
  WV_EUNSUPPORTED = -5   /* valid request the library does not implement */
} wv_status;

enum { WV_W53 = 0, WV_W97 = 1 };          /* wavelet: LeGall 5/3 integer, CDF 9/7 float32 */
enum { WV_GRAY8 = 0, WV_YUV420 = 1 };     /* plane format */
enum { WV_PATH_FUSED = 0, WV_PATH_PLAIN = 1 };

/* Stream geometry, fixed for the life of a context. */
typedef struct {
  int32_t width, height;  /* luma samples, multiples of tile */
  int32_t tile;           /* luma tile edge: power of two, 8 .. 1024 */
  int32_t levels;         /* L: decomposition levels per tile, 1 <= L, tile >> L >= 1
                             (YUV420: (tile/2) >> L >= 1) */
  int32_t wavelet;        /* WV_W53 or WV_W97 */
  int32_t format;         /* WV_GRAY8 (one plane) or WV_YUV420 (Y, Cb, Cr) */
} wv_desc;

/* One frame's stored coefficients (device, tile-major, Mallat order per tile).
 * 5/3: int16 quantisation indices, dequantised as c = qstep * q (Section 3.3's
 *      quantisation is inverted on decode; uniform step reading).
 * 9/7: float32 coefficient values, used as stored (qstep ignored). */
typedef struct {
  const void* planes[3];  /* [0] luma; [1], [2] Cb, Cr (NULL for WV_GRAY8) */
  int32_t frame_index;    /* position in the GOP; stamps record it */
  int32_t is_intra;       /* 1: rec = clip(P); 0: rec = clip(ref + P) (residual onto the previous frame) */
  int32_t qstep;          /* 5/3 dequantisation step, 1 .. 65535 */
  int32_t reserved;       /* must be 0 */
} wv_frame;

/* Reconstruction state of one stream (caller-owned).
 * planes: device, tile-major like the coefficients, uint8 (5/3) or float32
 * (9/7) samples in 0..255.  Read for residual frames and written for every
 * decoded tile: after a decode, the masked tiles hold rec of that frame.
 * tile_stamp: HOST array [n_tiles], the frame_index last reconstructed per
 * tile (-1 = none); checked and updated by the decode calls. */
typedef struct {
  void* planes[3];
  int32_t* tile_stamp;
} wv_ref;

typedef struct wv_ctx wv_ctx;

/* Create a decoding context on the current HIP device.  Allocates the
 * context's small device state (work counters) up front; decode calls never
 * allocate.  Errors: WV_EINVAL (bad geometry), WV_ENOMEM, WV_EDEVICE. */
wv_status wv_create(wv_ctx** ctx, const wv_desc* desc);

/* Release the context and its device memory (synchronises its device). */
wv_status wv_destroy(wv_ctx* ctx);

/* Static description of a status code. */
const char* wv_strerror(wv_status s);

/* Message of the last failing call on this host thread ("" if none). */
const char* wv_last_error(void);

/* Select the decode form used by wv_decode_viewport.
 * WV_PATH_FUSED (default): one launch per call, every step of the decode
 *   fused per output block (coefficient loads, all levels in LDS, residual,
 *   clip, colour).
 * WV_PATH_PLAIN: the per-step form -- gather/dequantise, one launch per
 *   level and direction, residual add + clip, colour -- through a workspace
 *   that this call allocates (8 bytes per coefficient of every tile).
 * Errors: WV_EINVAL, WV_ENOMEM. */
wv_status wv_set_path(wv_ctx* ctx, int32_t path);

/* Decode the viewport of one frame (Section 3.1: the inverse transform runs
 * only for the masked part of the frame).
 *  coeffs      : the frame's coefficients (device planes).
 *  level_count : HOST uint8 [n_tiles], detail levels applied per tile
 *                (0 .. levels); the finest levels - level_count[t] levels'
 *                detail bands are treated as zero and not read
 *                (foveated decoding, Section 3.7).  NULL = all levels.
 *  tile_mask   : HOST uint8 [n_tiles], nonzero = decode this tile.
 *  ref         : reconstruction state; for a residual frame every masked
 *                tile must have tile_stamp == frame_index - 1, else
 *                WV_ESTALE (replay the missing frames of those tiles first,
 *                with out = NULL).  On success the masked tiles' stamps
 *                become frame_index.
 *  out         : device, RGB of the masked tiles in ascending tile order,
 *                planar [n_visible][3][tile][tile] (WV_YUV420) or
 *                [n_visible][1][tile][tile] (WV_GRAY8: the luma itself);
 *                uint8 (5/3) or float32 clipped to [0, 255] (9/7).
 *                NULL = update ref only.
 *  stream      : HIP stream.
 * A mask with no tile set is valid and enqueues nothing. */
wv_status wv_decode_viewport(wv_ctx* ctx, const wv_frame* coeffs, const uint8_t* level_count,
                             const uint8_t* tile_mask, wv_ref* ref, void* out,
                             hipStream_t stream);

/* wv_decode_viewport for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context is needed and nothing is allocated.  desc gives the
 * geometry (as for wv_create); the other arguments, their layout, ownership,
 * the stamp rule and the errors are those of wv_decode_viewport.  The decode
 * runs in the first persistent fused variant that fits desc (WV_EUNSUPPORTED
 * if none); the only device memory it uses beyond the caller's buffers is a
 * fixed 256-byte array of this library per GPU (the work-queue counters of
 * the persistent kernels, cleared by a kernel at the start of each call and
 * kept until the process ends).  Every call on one GPU shares that array:
 * calls that overlap on one GPU (other streams, other host threads) race;
 * serialise them.  Tiles go in launches of at most 360. */
wv_status wv_decode_viewport_noalloc(const wv_desc* desc, const wv_frame* coeffs,
                                     const uint8_t* level_count, const uint8_t* tile_mask,
                                     wv_ref* ref, void* out, hipStream_t stream);

/* Consecutive frames of one viewport in one call (Section 3.1 per frame,
 * the residual chain of reading C5 across them): frames[f].frame_index must
 * be frames[0].frame_index + f; the same tile_mask and level_count apply to
 * every frame; the first frame obeys wv_decode_viewport's stamp rule.
 * outs: HOST array [n_frames] of device outputs (entries may be NULL), or
 * NULL.  With a row-strip variant the frames go in one launch (per group of
 * 8 frames): every tile strip is taken through the frames in order, so
 * workgroups need not wait for each other between frames.  Other forms
 * decode frame by frame.  On success the masked tiles' stamps become the
 * last frame's index.  Errors: as wv_decode_viewport. */
wv_status wv_decode_gop(wv_ctx* ctx, int32_t n_frames, const wv_frame* frames,
                        const uint8_t* level_count, const uint8_t* tile_mask, wv_ref* ref,
                        void* const* outs, hipStream_t stream);

/* ------------------------------------------------------ inter-frame sets
 * Section 3.2: n consecutive frames (n = 2 or 4 here; 4 in the paper's
 * experiments) form an inter-frame set.  Their frame-wise coefficients are
 * transformed once more along time, position by position, by the Haar
 * wavelet down to one approximation.  Reading of the normalisation: the
 * averaging form s = (a + b) / 2, d = (a - b) / 2, under which synthesis is
 * additions only, so frame t of a set is the approximation band plus one
 * signed detail band per level (log2 n additions):
 *   n = 4:  c_t = B0 + s1(t) * B1 + s0(t) * B[2 + t / 2]
 *   n = 2:  c_t = B0 + s0(t) * B1
 * where s1(t) = -1 if bit 1 of t is set, else +1, and s0(t) likewise for
 * bit 0.  Every frame of a set decodes on its own: no reference frame, no
 * stamps (the keyframe-free random access the paper motivates the sets with). */
typedef struct {
  const void* planes[3];  /* per plane: device bands [n][n_tiles][P][P] (each band
                             tile-major, Mallat order per tile, like a frame's
                             coefficients), in the order B0, B1, B2, B3.
                             5/3: int16 indices; 9/7: float32 values. */
  int32_t n;              /* frames per set: 2 or 4 */
  int32_t qstep[4];       /* 5/3: dequantisation step of each band, 1 .. 65535
                             (entries >= n ignored); 9/7: ignored */
} wv_set;

/* Decode frames t0 .. t0 + n_frames - 1 of an inter-frame set for one
 * viewport, in one launch: every visible coefficient is summed from its bands
 * as it is loaded (Section 3.2), then the inverse transform of Section 3.1
 * with the foveated level drop of Section 3.7, clip to 0..255 and colour,
 * exactly as wv_decode_viewport does for an intra frame of coefficients c_t.
 * 5/3 sums and lifting run in 32-bit integers (exact while they fit).
 *  level_count, tile_mask : as for wv_decode_viewport.
 *  outs : HOST array [n_frames] of device outputs, none NULL, each laid out
 *         like wv_decode_viewport's out.
 * Needs a row-strip geometry (tile 512, 3 .. 5 levels): the fused row-strip
 * kernel of the context's variant runs (the 4-wave grid form of its shape).
 * Errors: WV_EINVAL (arguments, t0 / n_frames outside the set),
 * WV_EUNSUPPORTED (geometry without row strips, n not 2 or 4), WV_EDEVICE. */
wv_status wv_decode_set(wv_ctx* ctx, const wv_set* set, int32_t t0, int32_t n_frames,
                        const uint8_t* level_count, const uint8_t* tile_mask, void* const* outs,
                        hipStream_t stream);

/* One viewport decode inside a batch. */
typedef struct {
  wv_ctx* ctx;
  const wv_frame* coeffs;
  const uint8_t* level_count;
  const uint8_t* tile_mask;
  wv_ref* ref;
  void* out;
} wv_job;

/* Fused form over uneven tile sets (Section 3.5: the decode of the visible
 * regions overlaps other work instead of running pass by pass; Section 3.1
 * per viewport): all jobs (one or many viewports, of the same or different
 * streams, with their own masks and level counts) decoded by a single
 * launch that takes (tile, strip or block) work units from the job and item
 * tables -- in the kernel arguments up to 360 visible tiles, beyond that in
 * the context's device table, filled stream-ordered from pinned staging --
 * with the launch shape the context's tuner picked.  Every job obeys
 * wv_decode_viewport's rules; all contexts must be on the current device and
 * share tile, levels, wavelet and format (else WV_EUNSUPPORTED).  Two jobs
 * may not write the same ref tile.  All-or-nothing: on error no job runs and
 * no stamp changes.  At most 256 jobs and 65536 visible tiles per call. */
wv_status wv_decode_batch(int32_t n_jobs, const wv_job* jobs, hipStream_t stream);

/* Viewport tile selection from a head pose (Sections 3.1 and 3.6): the frame
 * is top-bottom stereo, each eye an equirectangular width x height/2 image.
 * A tile is selected when any of samples x samples points inside it (at
 * (j + 0.5) * tile / samples) maps to a direction inside the rectilinear
 * fov_h x fov_v (degrees) frustum around (yaw, pitch) (degrees).  eyes = 1:
 * top eye only; 2: both eyes with the same pose.  mask: HOST uint8 [n_tiles].
 * Host only, float64.  Errors: WV_EINVAL. */
wv_status wv_viewport_mask(const wv_desc* desc, double yaw, double pitch, double fov_h,
                           double fov_v, int32_t samples, int32_t eyes, uint8_t* mask);

/* Foveated level counts (Section 3.7): per tile, the angle between the gaze
 * (yaw, pitch) and the tile-centre direction; levels - 0 within inner
 * degrees, levels - 1 within outer degrees, levels - 2 beyond (not below 0).
 * level_count: HOST uint8 [n_tiles].  Errors: WV_EINVAL. */
wv_status wv_foveation_levels(const wv_desc* desc, double yaw, double pitch, double inner,
                              double outer, uint8_t* level_count);

/* Encode source planes into stored intra coefficients (the forward
 * transform of Section 3.1 per tile -- every column then every row per
 * level -- and the uniform quantiser q = sign(c) floor(|c|/qstep + 1/2)).
 * src: device tile-major uint8 planes; coeffs: device tile-major planes,
 * int16 indices (5/3) or float32 values qstep*q (9/7, computed in float64).
 * Allocates and frees a temporary workspace (not for hot loops).
 * Errors: WV_EINVAL (NULL planes, qstep < 1, an index outside int16),
 * WV_ENOMEM, WV_EDEVICE. */
wv_status wv_encode_intra(wv_ctx* ctx, const void* const* src, void* const* coeffs,
                          int32_t qstep, hipStream_t stream);

/* Autotuner: times every compiled fused-kernel variant (block shape, threads,
 * grid form) on a synthetic decode of n_visible tiles of this context's
 * geometry (scratch buffers allocated and freed here), keeps the fastest for
 * the context and returns its index.  reps >= 1 timed launches per variant.
 * Errors: WV_EINVAL, WV_ENOMEM, WV_EDEVICE. */
wv_status wv_autotune(wv_ctx* ctx, int32_t n_visible, int32_t reps, hipStream_t stream,
                      int32_t* best_variant);

/* Number of fused variants, and the one in use; select one by index. */
int32_t wv_variant_count(const wv_ctx* ctx);
wv_status wv_get_variant(const wv_ctx* ctx, int32_t* variant);
wv_status wv_set_variant(wv_ctx* ctx, int32_t variant);

/* Human-readable description of a variant (static string). */
const char* wv_variant_name(const wv_ctx* ctx, int32_t variant);

/* ------------------------------------------------------------------ serving
 * Many head-tracked streams decoded together (Section 3.1: each client's
 * viewport is decoded from the shared stored coefficients; Section 3.6:
 * selection follows the head pose; Section 3.7: optional foveation).
 * A server owns one slot per admitted stream -- the stream's reconstruction
 * planes for every tile plus one frame of output -- and as many slots as
 * max_active and the HBM budget allow.  wv_server_run plays the added
 * streams: a stream is admitted when a slot is free (in the order added),
 * each of its frames is requested at its arrival time, and every turn of
 * the loop decodes the next frame of every stream whose request has
 * arrived, all in one persistent fused launch (a replayed HIP graph; tiles
 * that enter a viewport after a missed frame have the missing frames of
 * their GOP replayed first, in launches of their own).  Results are those
 * of wv_decode_viewport on each stream alone: the decode of a tile depends
 * only on its own coefficients, reference and level count. */
typedef struct wv_server wv_server;

/* How a client views the frame. */
typedef struct {
  double fov_h, fov_v;     /* rectilinear field of view, degrees, (0, 180) */
  int32_t eyes;            /* 1: top eye only; 2: both eyes, same pose */
  int32_t foveate;         /* 0: all levels; 1: wv_foveation_levels(inner, outer) */
  double inner, outer;     /* foveation eccentricities, degrees */
} wv_view_class;

/* One client stream.  Host arrays are copied by wv_server_add_stream. */
typedef struct {
  int32_t source;          /* sources are numbered 0, 1, ... in the order added */
  int32_t n_frames;        /* frame t plays source frame t mod gop_len */
  const double* arrival;   /* HOST [n_frames] request times, seconds, >= 0, non-decreasing */
  const double* yaw;       /* HOST [n_frames] head pose per frame, degrees */
  const double* pitch;     /* HOST [n_frames] */
  wv_view_class view;      /* tile samples per edge: 16 */
  void* const* out_frames; /* HOST [n_frames] device outputs laid out as wv_decode_viewport's
                              out (room for max_visible tiles), or NULL: the slot's own buffer,
                              overwritten every frame */
} wv_stream_desc;

typedef struct {
  int64_t requests;        /* frames requested over all streams */
  int64_t frames_decoded;
  int64_t tiles_decoded;   /* visible tiles of requested frames */
  int64_t catchup_tiles;   /* tiles replayed for missed frames */
  int64_t launches;        /* persistent-kernel launches */
  int64_t turns;           /* loop turns that enqueued work */
  int64_t admitted;        /* streams admitted */
  int64_t max_active;      /* most streams holding a slot at once */
  double mpix;             /* output megapixels (luma samples of visible tiles) */
  double wall_s;           /* host time of the run */
  double gpu_ms;           /* GPU time from start to the last completion */
  double p50_ms, p99_ms, max_ms, mean_ms;   /* request latency: completion - arrival */
} wv_server_stats;

/* Create a server for one frame geometry.  max_active: 1..256 slots wanted;
 * hbm_budget: device bytes the slots may take (the slot count is
 * min(max_active, budget / slot bytes)); max_visible: most visible tiles per
 * frame.  The persistent variant is the first that fits the geometry.
 * Errors: WV_EINVAL, WV_ENOMEM (budget below one slot, or allocation),
 * WV_EUNSUPPORTED (no persistent variant fits), WV_EDEVICE. */
wv_status wv_server_create(wv_server** srv, const wv_desc* desc, int32_t max_active,
                           int64_t hbm_budget, int32_t max_visible);
wv_status wv_server_destroy(wv_server* srv);

/* Slots the budget allowed (0 for NULL). */
int32_t wv_server_slots(const wv_server* srv);

/* Register a GOP of device coefficient frames (frame 0 intra, the rest
 * residual; planes as in wv_decode_viewport); the caller keeps them alive
 * while the server runs.  Errors: WV_EINVAL. */
wv_status wv_server_add_source(wv_server* srv, int32_t gop_len, const wv_frame* frames);

/* Queue a stream for the next wv_server_run.  Errors: WV_EINVAL. */
wv_status wv_server_add_stream(wv_server* srv, const wv_stream_desc* stream);

/* Forget the queued streams (sources stay). */
wv_status wv_server_clear_streams(wv_server* srv);

/* Play every queued stream to its end on HIP stream `stream`.  time_scale:
 * wall seconds per second of arrival time (1 = real time; 0 = every request
 * arrives at the start, for throughput).  latency_ms: HOST [total requests]
 * or NULL, in stream order then frame order.  Blocks until all work is
 * done.  Errors: WV_EINVAL, WV_EUNSUPPORTED (a viewport above max_visible),
 * WV_EDEVICE. */
wv_status wv_server_run(wv_server* srv, double time_scale, double* latency_ms,
                        wv_server_stats* stats, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* WV_H */
