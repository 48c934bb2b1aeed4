// Internal types shared by the HIP kernels and the host side of libwv.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wv.h"

namespace wv {

// One viewport decode as the kernels see it (64 bytes).
struct Job {
  const void* coef[3];   // coefficient planes (tile-major); inter-frame set: band 0
  void* ref[3];          // reconstruction planes (tile-major), read for residual frames
                         // (NULL for inter-frame-set frames: no reference is kept)
  void* out;             // RGB / grey output, [n_visible][C][tile][tile]
  int32_t qstep;         // 5/3 dequantisation step (set: step of band 0)
  uint32_t flags;        // kJobIntra | kJobHasOut
  // Inter-frame-set frames only (strip kernels compiled for sets): the
  // frame's coefficients are band 0 + hq[0] * band 1 + hq[1] * band hband,
  // bands hstride luma elements apart (chroma: hstride / 4).  hq are signed
  // steps (5/3) or signs (9/7); hq[1] = 0 for sets of two.
  uint32_t hstride;
  uint32_t hband;
  int32_t hq[2];
};
constexpr uint32_t kJobIntra = 1u;
constexpr uint32_t kJobHasOut = 2u;

// One visible tile of one job (8 bytes).
struct Item {
  uint16_t tile;   // tile index inside the job's frame
  uint16_t slot;   // position of the tile in the job's output (ascending tile order)
  uint8_t job;     // index into the job table
  uint8_t lc;      // detail levels applied (levels - dropped)
  uint16_t pad;
};

constexpr int kArgJobs = 8;
constexpr int kArgItems = 360;

// Work description passed by value in the kernel-argument segment.  When the
// work does not fit, jobs/items live in device memory (jobs_dev/items_dev).
struct WorkArgs {
  int32_t n_items;
  int32_t tile;          // luma tile edge
  int32_t levels;
  int32_t bx, by;        // luma blocks per tile in x and y
  int32_t total;         // n_items * bx * by work units
  uint32_t* counter;     // persistent form: [0] next unit, [1] finished groups
  const int32_t* total_dev;  // when non-null, the unit count is read here (graph replays)
  int32_t n_frames;      // > 0: every unit decodes its tile for jobs 0 .. n_frames-1 in order
                         // (one viewport's consecutive frames; strip kernels only)
  const Job* jobs_dev;
  const Item* items_dev;
  Job jobs[kArgJobs];
  Item items[kArgItems];
};

static_assert(sizeof(WorkArgs) <= 4000, "kernel arguments must stay under 4 KB");

// Plain path: per-step kernels over a workspace (4 bytes per coefficient).
struct PlainArgs {
  int32_t n_items;
  int32_t tile;
  int32_t levels;
  int32_t nplanes;
  int32_t qstep;
  uint32_t flags;
  const void* coef[3];
  void* ref[3];
  void* out;
  void* ws;              // [n_items][planes] tile-planes of int32 / float
  Item items[256];
};
static_assert(sizeof(PlainArgs) <= 4000, "kernel arguments must stay under 4 KB");

// Fused variants (block shape, threads, grid form).
struct Variant {
  const char* name;
  int bw, bh, nt;
  bool persistent;
  int groups_per_cu;     // persistent form: resident groups per CU
  bool general;          // handles mirrored regions smaller than 16 samples
  int levels;            // fast and strip variants: the level count they are compiled for (0 = any)
  int shape;             // fast and strip variants: shape index in their launcher
  int kind;              // 0 block (runtime level count), 1 fast block, 2 row strip
  int format;            // the only format it is built for, or -1 for both
  int wavelet;           // the only wavelet it is built for, or -1 for both
};

// Launchers (wv_kernels.hip).  Return hipSuccess or the launch error.
int fused_variant_count(int wavelet, int format);
const Variant* fused_variant(int wavelet, int format, int v);
hipError_t launch_fused(int wavelet, int format, int v, const WorkArgs& a, int n_cu,
                        hipStream_t s);
hipError_t launch_fast53(int format, int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                         hipStream_t s);
hipError_t launch_fast97(int format, int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                         hipStream_t s);
hipError_t launch_strip53(int format, int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                          hipStream_t s);
hipError_t launch_strip97(int format, int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                          hipStream_t s);
// Inter-frame-set frames (jobs with the hstride / hband / hq fields), grid form.
hipError_t launch_strip53_set(int format, int shape, int L, const WorkArgs& a, hipStream_t s);
hipError_t launch_strip97_set(int format, int shape, int L, const WorkArgs& a, hipStream_t s);
hipError_t launch_plain(int wavelet, int format, const PlainArgs& a, hipStream_t s);

// Rebuild of dense planes from the sparse format: one workgroup per (visible
// tile, block) of one plane.
constexpr int kRebuildMaxBlocks = 256;   // blocks per tile (512-sample tiles)
struct RebuildArgs {
  const uint32_t* block_end;
  const uint8_t* values;
  const uint16_t* index;
  uint64_t n_records;
  void* dense;                           // [n_tiles][P][P] int16 or float32
  int32_t p, levels, b, nb;              // tile edge, levels, block edge, blocks per tile
  float lo[2], scale[2];                 // [0] approximation, [1] details
  int32_t n_items;
  int32_t compact;                       // block_end indexed by item slot (staged
                                         // records of the visible tiles only)
  uint16_t order[kRebuildMaxBlocks];     // storage order: (by << 8) | bx
  Item items[kArgItems];
};
static_assert(sizeof(RebuildArgs) <= 4000, "kernel arguments must stay under 4 KB");
hipError_t launch_rebuild(int wavelet, const RebuildArgs& a, hipStream_t s);
hipError_t launch_encode(int wavelet, int nplanes, int n_tiles, int tile, int levels,
                         int qstep, const void* const* src, void* const* dst, void* ws,
                         int* overflow_flag, hipStream_t s);

}  // namespace wv
