// The sparse storage format (Sections 3.3, 3.4, 3.6): host encoder, and the
// entry point of the GPU rebuild (Section 3.5).  The encoder is offline work,
// as in the paper: plain host code, one plane of one frame per call.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "wv_ctx.h"
#include "wv_format.h"

using namespace wv;
using namespace wvp;

namespace {

int block_edge(int p) { return std::min(32, p); }

// Level of the detail region that holds position (y, x) of a P x P Mallat
// plane: k for the level-k detail bands (1 = finest), 0 for the approximation.
int position_level(int p, int levels, int y, int x) {
  const int m = std::max(y, x);
  int lev = 0;
  for (int k = levels; k >= 1; --k)
    if (m >= (p >> k)) lev = k;
  return lev;
}

// Level of a block: that of its origin's region, levels + 1 for the block
// holding the approximation.
int block_level(int p, int levels, int by, int bx) {
  const int lev = position_level(p, levels, by * block_edge(p), bx * block_edge(p));
  return lev == 0 ? levels + 1 : lev;
}

// Blocks of a tile in storage order: by level from the lowest frequency,
// row-major within a level.
std::vector<std::pair<int, int>> storage_order(int p, int levels) {
  const int nbx = p / block_edge(p);
  std::vector<std::pair<int, int>> order;
  for (int by = 0; by < nbx; ++by)
    for (int bx = 0; bx < nbx; ++bx) order.emplace_back(by, bx);
  std::stable_sort(order.begin(), order.end(), [&](const auto& u, const auto& v) {
    return block_level(p, levels, u.first, u.second) > block_level(p, levels, v.first, v.second);
  });
  return order;
}

// Blocks of a tile kept at each level count lc = 0 .. levels: those whose
// level exceeds levels - lc, a prefix of the storage order.
std::vector<int> kept_table(int p, int levels) {
  std::vector<int> kept(levels + 1, 0);
  for (const auto& b : storage_order(p, levels)) {
    const int lev = block_level(p, levels, b.first, b.second);
    for (int lc = 0; lc <= levels; ++lc) kept[lc] += lev > levels - lc;
  }
  return kept;
}

bool plane_geometry(const wv_desc* d, int plane, int& p, int& height, int& tiles_x, int& n_tiles) {
  if (!d || d->tile < 8 || d->width % d->tile || d->height % d->tile) return false;
  const int nplanes = d->format == WV_YUV420 ? 3 : 1;
  if (plane < 0 || plane >= nplanes) return false;
  p = plane == 0 ? d->tile : d->tile / 2;
  height = plane == 0 ? d->height : d->height / 2;
  tiles_x = d->width / d->tile;
  n_tiles = tiles_x * (d->height / d->tile);
  return d->levels >= 1 && (p >> d->levels) >= 1;
}

}  // namespace

extern "C" int32_t wv_sparse_blocks_per_tile(const wv_desc* d, int32_t plane) {
  int p, h, tx, nt;
  if (!plane_geometry(d, plane, p, h, tx, nt)) return 0;
  const int n = p / block_edge(p);
  return n * n;
}

extern "C" wv_status wv_sparse_encode_plane(const wv_desc* d, int32_t plane, const float* coef,
                                            double alpha, int32_t poles, uint32_t* block_end,
                                            uint8_t* values, uint16_t* index, int64_t* n_records,
                                            float* bounds) {
  int p, height, tiles_x, n_tiles;
  if (!plane_geometry(d, plane, p, height, tiles_x, n_tiles))
    return fail(WV_EINVAL, "wv_sparse_encode_plane: bad geometry or plane %d", plane);
  if (!coef || !block_end || !values || !index || !n_records || !bounds)
    return fail(WV_EINVAL, "wv_sparse_encode_plane: NULL argument");
  if (!(alpha >= 0.0) || !std::isfinite(alpha))
    return fail(WV_EINVAL, "wv_sparse_encode_plane: alpha must be finite and >= 0");
  const int L = d->levels, b = block_edge(p);
  const size_t pp = (size_t)p * p;
  if ((size_t)n_tiles * pp > 0xffffffffull)
    return fail(WV_EINVAL, "wv_sparse_encode_plane: more coefficients than 32-bit block ends address");
  // per position of a tile: level, and the centre row of the samples it covers
  std::vector<int> lev(pp);
  std::vector<double> centre(pp);
  for (int y = 0; y < p; ++y)
    for (int x = 0; x < p; ++x) {
      const int k = position_level(p, L, y, x);
      lev[(size_t)y * p + x] = k;
      if (k == 0) {
        centre[(size_t)y * p + x] = (y + 0.5) * (double)(1 << L);
      } else {
        const int half = p >> k;
        const int band_row = y >= half ? y - half : y;
        centre[(size_t)y * p + x] = (band_row + 0.5) * (double)(1 << k);
      }
    }
  // Eq. 3 level weights, l = k - 1, l_max = L
  std::vector<double> lw(L + 1, 0.0);
  for (int k = 1; k <= L; ++k) {
    const double w = (double)(L - (k - 1)) / L;
    lw[k] = w * w;
  }
  const double eye = height / 2.0;
  const double pi = 3.14159265358979323846;
  // pass 1: keep decisions (Eq. 2) and the Eq. 4 bounds of the kept values
  std::vector<uint8_t> keep((size_t)n_tiles * pp);
  float amin = 0, amax = 0, dmin = 0, dmax = 0;
  bool any_a = false, any_d = false;
  for (int t = 0; t < n_tiles; ++t) {
    const double row0 = (double)(t / tiles_x) * p;
    for (size_t i = 0; i < pp; ++i) {
      const float c = coef[(size_t)t * pp + i];
      bool k;
      if (lev[i] == 0) {
        k = true;
        if (!any_a) { amin = amax = c; any_a = true; }
        amin = std::min(amin, c);
        amax = std::max(amax, c);
      } else if (c == 0.0f) {
        k = false;                // thresholds are never negative
      } else {
        const double h = poles ? 1.0 - std::sin(pi * std::fmod(row0 + centre[i], eye) / eye) : 0.0;
        const double thr = alpha * lw[lev[i]] + h;
        k = std::fabs((double)c) / 255.0 > thr;
        if (k) {
          if (!any_d) { dmin = dmax = c; any_d = true; }
          dmin = std::min(dmin, c);
          dmax = std::max(dmax, c);
        }
      }
      keep[(size_t)t * pp + i] = k;
    }
  }
  bounds[0] = amin;
  bounds[1] = amax;
  bounds[2] = dmin;
  bounds[3] = dmax;
  // pass 2: records, block by block in storage order (Eq. 4 codes)
  const auto order = storage_order(p, L);
  const int nb = (int)order.size();
  const int ap = p >> L;
  int64_t r = 0;
  for (int t = 0; t < n_tiles; ++t) {
    for (int j = 0; j < nb; ++j) {
      const int by = order[j].first, bx = order[j].second;
      for (int yy = 0; yy < b; ++yy)
        for (int xx = 0; xx < b; ++xx) {
          const int y = by * b + yy, x = bx * b + xx;
          const size_t i = (size_t)t * pp + (size_t)y * p + x;
          if (!keep[i]) continue;
          const bool is_a = y < ap && x < ap;
          const double lo = is_a ? amin : dmin, hi = is_a ? amax : dmax;
          const double span = hi - lo;
          const double code = span > 0 ? std::floor(((double)coef[i] - lo) / span * 255.0 + 0.5) : 0.0;
          values[r] = (uint8_t)code;
          index[r] = (uint16_t)(yy * b + xx);
          ++r;
        }
      block_end[(size_t)t * nb + j] = (uint32_t)r;
    }
  }
  *n_records = r;
  return WV_OK;
}

extern "C" wv_status wv_sparse_rebuild(wv_ctx* c, const wv_sparse_plane* planes, const uint8_t* lc,
                                       const uint8_t* mask, void* const* dense, hipStream_t s) {
  if (!c || !planes || !mask || !dense) return fail(WV_EINVAL, "wv_sparse_rebuild: NULL argument");
  for (int p = 0; p < c->nplanes; ++p) {
    const wv_sparse_plane& sp = planes[p];
    if (!sp.block_end || !dense[p] || sp.n_records < 0 || (sp.n_records > 0 && (!sp.values || !sp.index)))
      return fail(WV_EINVAL, "wv_sparse_rebuild: plane %d: missing arrays", p);
    if (!aligned16(dense[p])) return fail(WV_EINVAL, "wv_sparse_rebuild: dense[%d] is not 16-byte aligned", p);
    if (wv_sparse_blocks_per_tile(&c->d, p) > kRebuildMaxBlocks)
      return fail(WV_EUNSUPPORTED, "wv_sparse_rebuild: tiles above 512 samples");
  }
  std::vector<Item> items;
  for (int t = 0; t < c->n_tiles; ++t) {
    if (!mask[t]) continue;
    const int l = lc ? lc[t] : c->d.levels;
    if (l > c->d.levels)
      return fail(WV_EINVAL, "wv_sparse_rebuild: level_count[%d] = %d exceeds levels %d", t, l, c->d.levels);
    Item it = {};
    it.tile = (uint16_t)t;
    it.slot = (uint16_t)items.size();
    it.lc = (uint8_t)l;
    items.push_back(it);
  }
  for (int p = 0; p < c->nplanes; ++p) {
    const wv_sparse_plane& sp = planes[p];
    RebuildArgs a;
    memset(&a, 0, sizeof a);
    a.block_end = sp.block_end;
    a.values = sp.values;
    a.index = sp.index;
    a.n_records = (uint64_t)sp.n_records;
    a.dense = dense[p];
    a.p = plane_edge(c->d, p);
    a.levels = c->d.levels;
    a.b = block_edge(a.p);
    const auto order = storage_order(a.p, a.levels);
    a.nb = (int)order.size();
    for (int j = 0; j < a.nb; ++j) a.order[j] = (uint16_t)((order[j].first << 8) | order[j].second);
    for (int k = 0; k < 2; ++k) {
      const double lo = sp.bounds[2 * k], hi = sp.bounds[2 * k + 1];
      a.lo[k] = (float)lo;
      a.scale[k] = (float)((hi - lo) / 255.0);
    }
    for (size_t i0 = 0; i0 < items.size(); i0 += kArgItems) {
      const int n = (int)std::min<size_t>(kArgItems, items.size() - i0);
      std::copy(items.begin() + i0, items.begin() + i0 + n, a.items);
      a.n_items = n;
      const hipError_t e = launch_rebuild(c->d.wavelet, a, s);
      if (e != hipSuccess) return hip_fail(e, "rebuild launch");
    }
  }
  return WV_OK;
}

namespace {

// Record range of each visible tile of one plane: [begin, end) in the plane's
// record arrays, and the tile's block ends (clamped to n_records) from which
// the staged table is made.
struct TileRun {
  int64_t begin, end;
  int kept;   // blocks kept
};

// kept: kept_table of the plane's tile edge
wv_status tile_runs(const wv_desc* d, int plane, const std::vector<int>& kept, const uint32_t* block_end,
                    int64_t n_records, const uint8_t* lc, const uint8_t* mask, std::vector<TileRun>& out) {
  int p, height, tiles_x, n_tiles;
  if (!plane_geometry(d, plane, p, height, tiles_x, n_tiles))
    return fail(WV_EINVAL, "record runs: bad geometry or plane %d", plane);
  if (!block_end || !mask) return fail(WV_EINVAL, "record runs: NULL block_end or tile_mask");
  if (n_records < 0) return fail(WV_EINVAL, "record runs: negative record count");
  const int nb = (p / block_edge(p)) * (p / block_edge(p));
  out.clear();
  for (int t = 0; t < n_tiles; ++t) {
    if (!mask[t]) continue;
    const int l = lc ? lc[t] : d->levels;
    if (l > d->levels) return fail(WV_EINVAL, "level_count[%d] = %d exceeds levels %d", t, l, d->levels);
    const size_t g0 = (size_t)t * nb;
    int64_t prev = t ? std::min<int64_t>(block_end[g0 - 1], n_records) : 0;
    const int64_t begin = prev;
    for (int j = 0; j < kept[l]; ++j) {
      const int64_t e = std::min<int64_t>(block_end[g0 + j], n_records);
      if (e < prev) return fail(WV_EINVAL, "block ends of tile %d decrease at block %d", t, j);
      prev = e;
    }
    out.push_back({begin, prev, kept[l]});
  }
  return WV_OK;
}

}  // namespace

extern "C" wv_status wv_sparse_visible_runs(const wv_desc* d, int32_t plane, const uint32_t* block_end,
                                            int64_t n_records, const uint8_t* lc, const uint8_t* mask,
                                            int64_t* run_begin, int64_t* run_end, int32_t* n_runs,
                                            int64_t* n_in_runs) {
  if (!run_begin || !run_end || !n_runs || !n_in_runs) return fail(WV_EINVAL, "wv_sparse_visible_runs: NULL output");
  int p, height, tiles_x, n_tiles;
  if (!plane_geometry(d, plane, p, height, tiles_x, n_tiles))
    return fail(WV_EINVAL, "wv_sparse_visible_runs: bad geometry or plane %d", plane);
  std::vector<TileRun> tr;
  const wv_status st = tile_runs(d, plane, kept_table(p, d->levels), block_end, n_records, lc, mask, tr);
  if (st != WV_OK) return st;
  int n = 0;
  int64_t total = 0;
  for (const TileRun& r : tr) {
    if (r.end == r.begin) continue;
    total += r.end - r.begin;
    if (n > 0 && run_end[n - 1] == r.begin) {
      run_end[n - 1] = r.end;
    } else {
      run_begin[n] = r.begin;
      run_end[n] = r.end;
      ++n;
    }
  }
  *n_runs = n;
  *n_in_runs = total;
  return WV_OK;
}

// ---------------------------------------------------------------------------
// Prefetcher (Section 3.5, Fig. 4)
//
// wv_prefetch_stage checks a set and lays out its slot in the caller's
// thread, then hands the work that takes time -- waiting for the slot's
// pinned buffer, gathering the record runs into it, enqueueing the upload --
// to the prefetcher's own thread (the paper's prepare thread), so that the
// caller goes on enqueueing GPU work meanwhile.  wv_prefetch_rebuild waits
// (on the host) until its slot's upload is enqueued.

namespace {

constexpr int kPrefetchSlots = 2;
constexpr int kPrefetchMaxFrames = 16;

size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// One frame-plane of a staged set: offsets into the slot, records, bounds.
struct StagedPlane {
  size_t be_off, idx_off, val_off;
  int64_t n;
  float bounds[4];
};

struct Slot {
  bool staged = false;      // staged and not yet rebuilt
  bool ready = false;       // its upload is enqueued (or failed: err)
  bool copied_rec = false, consumed_rec = false;
  wv_status err = WV_OK;
  char msg[160] = {};
  int n_frames = 0;
  std::vector<Item> items;
  std::vector<StagedPlane> planes;
};

// The prepare thread's work for one set.
struct StageJob {
  int k = 0;
  bool direct = false;
  int n_vis = 0;
  size_t bytes = 0;                         // slot bytes in use
  std::vector<wv_sparse_plane> frames;      // [n_frames * nplanes], the caller's store
  std::vector<std::vector<TileRun>> runs;
  std::vector<StagedPlane> planes;
  std::vector<Item> items;
};

}  // namespace

struct wv_prefetch {
  wv_ctx* ctx = nullptr;
  int max_frames = 0;
  size_t cap = 0;
  hipStream_t copy = nullptr;
  unsigned char* host[kPrefetchSlots] = {};
  unsigned char* dev[kPrefetchSlots] = {};
  hipEvent_t copied[kPrefetchSlots] = {};    // the slot's upload has finished
  hipEvent_t consumed[kPrefetchSlots] = {};  // the slot's rebuild has finished
  Slot slot[kPrefetchSlots];
  int next_stage = 0, next_rebuild = 0;
  std::vector<int> kept[3];                    // kept_table of each plane
  std::vector<uint16_t> order[3];              // storage order of each plane
  // the prepare thread
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<StageJob> jobs;
  bool quit = false;
};

namespace {

// Gather and upload of one staged set (prepare thread).  Returns the HIP
// error, if any, with what failed in `what`.
hipError_t run_stage_job(wv_prefetch* pf, StageJob& j, const char** what) {
  const wv_ctx* c = pf->ctx;
  const int np = c->nplanes, nfp = (int)j.frames.size(), k = j.k;
  bool copied_rec, consumed_rec;
  {
    std::lock_guard<std::mutex> lock(pf->mu);
    copied_rec = pf->slot[k].copied_rec;
    consumed_rec = pf->slot[k].consumed_rec;
  }
  *what = "wait for the slot";
  // the pinned buffer is free once its previous upload has finished
  hipError_t e = copied_rec ? hipEventSynchronize(pf->copied[k]) : hipSuccess;
  if (e != hipSuccess) return e;
  unsigned char* h = pf->host[k];
  for (int i = 0; i < nfp; ++i) {
    const wv_sparse_plane& sp = j.frames[i];
    const StagedPlane& s = j.planes[i];
    const int p = i % np, nb = wv_sparse_blocks_per_tile(&c->d, p);
    uint32_t* be = (uint32_t*)(h + s.be_off);
    int64_t cur = 0;   // staged records so far
    for (size_t v = 0; v < j.runs[i].size(); ++v) {
      const TileRun& r = j.runs[i][v];
      const int t = j.items[v].tile, kb = r.kept;
      for (int b = 0; b < nb; ++b) {
        const int64_t end = b < kb ? std::min<int64_t>(sp.block_end[(size_t)t * nb + b], sp.n_records) : r.end;
        be[(size_t)v * nb + b] = (uint32_t)(cur + (end - r.begin));
      }
      if (!j.direct && r.end > r.begin) {
        std::memcpy(h + s.idx_off + (size_t)cur * 2, sp.index + r.begin, (size_t)(r.end - r.begin) * 2);
        std::memcpy(h + s.val_off + (size_t)cur, sp.values + r.begin, (size_t)(r.end - r.begin));
      }
      cur += r.end - r.begin;
    }
  }
  *what = "upload";
  // after the slot's previous rebuild has read the device copy
  if (consumed_rec) e = hipStreamWaitEvent(pf->copy, pf->consumed[k], 0);
  if (e == hipSuccess && j.bytes > 0) {
    if (!j.direct) {
      e = hipMemcpyAsync(pf->dev[k], h, j.bytes, hipMemcpyHostToDevice, pf->copy);
    } else {
      for (int i = 0; e == hipSuccess && i < nfp; ++i) {
        const wv_sparse_plane& sp = j.frames[i];
        const StagedPlane& s = j.planes[i];
        const int nb = wv_sparse_blocks_per_tile(&c->d, i % np);
        e = hipMemcpyAsync(pf->dev[k] + s.be_off, h + s.be_off, (size_t)j.n_vis * nb * 4, hipMemcpyHostToDevice,
                           pf->copy);
        int64_t cur = 0;
        for (size_t v = 0; e == hipSuccess && v < j.runs[i].size(); ++v) {
          // a run of tiles whose records touch is one copy per array
          const int64_t b0 = j.runs[i][v].begin, c0 = cur;
          int64_t e0 = j.runs[i][v].end;
          while (v + 1 < j.runs[i].size() && j.runs[i][v + 1].begin == e0) e0 = j.runs[i][++v].end;
          const size_t n = (size_t)(e0 - b0);
          cur += (int64_t)n;
          if (!n) continue;
          e = hipMemcpyAsync(pf->dev[k] + s.idx_off + (size_t)c0 * 2, sp.index + b0, n * 2, hipMemcpyHostToDevice,
                             pf->copy);
          if (e == hipSuccess)
            e = hipMemcpyAsync(pf->dev[k] + s.val_off + (size_t)c0, sp.values + b0, n, hipMemcpyHostToDevice,
                               pf->copy);
        }
      }
    }
  }
  if (e == hipSuccess) e = hipEventRecord(pf->copied[k], pf->copy);
  return e;
}

void prepare_thread(wv_prefetch* pf) {
  const bool dev_ok = hipSetDevice(pf->ctx->device) == hipSuccess;
  for (;;) {
    StageJob j;
    {
      std::unique_lock<std::mutex> lock(pf->mu);
      pf->cv.wait(lock, [&] { return pf->quit || !pf->jobs.empty(); });
      if (pf->jobs.empty()) return;   // quit with nothing left
      j = std::move(pf->jobs.front());
      pf->jobs.pop_front();
    }
    const char* what = "set the device";
    const hipError_t e = dev_ok ? run_stage_job(pf, j, &what) : hipErrorInvalidDevice;
    {
      std::lock_guard<std::mutex> lock(pf->mu);
      Slot& sl = pf->slot[j.k];
      sl.ready = true;
      sl.copied_rec = sl.copied_rec || e == hipSuccess;
      sl.err = e == hipSuccess ? WV_OK : WV_EDEVICE;
      if (e != hipSuccess)
        std::snprintf(sl.msg, sizeof sl.msg, "wv_prefetch_stage: %s: %s", what, hipGetErrorString(e));
    }
    pf->cv.notify_all();
  }
}

}  // namespace

extern "C" wv_status wv_prefetch_destroy(wv_prefetch* pf) {
  if (!pf) return WV_OK;
  if (pf->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lock(pf->mu);
      pf->quit = true;
    }
    pf->cv.notify_all();
    pf->worker.join();   // finishes the jobs already handed to it
  }
  hipSetDevice(pf->ctx->device);
  if (pf->copy) hipStreamSynchronize(pf->copy);
  for (int k = 0; k < kPrefetchSlots; ++k) {
    if (pf->consumed[k]) {
      if (pf->slot[k].consumed_rec) hipEventSynchronize(pf->consumed[k]);
      hipEventDestroy(pf->consumed[k]);
    }
    if (pf->copied[k]) hipEventDestroy(pf->copied[k]);
    if (pf->host[k]) hipHostFree(pf->host[k]);
    if (pf->dev[k]) hipFree(pf->dev[k]);
  }
  if (pf->copy) hipStreamDestroy(pf->copy);
  delete pf;
  return WV_OK;
}

extern "C" wv_status wv_prefetch_create(wv_ctx* c, int32_t max_frames, int64_t slot_bytes, wv_prefetch** out) {
  if (!out) return fail(WV_EINVAL, "wv_prefetch_create: NULL out-pointer");
  *out = nullptr;
  if (!c) return fail(WV_EINVAL, "wv_prefetch_create: NULL context");
  if (max_frames < 1 || max_frames > kPrefetchMaxFrames)
    return fail(WV_EINVAL, "wv_prefetch_create: max_frames %d outside 1 .. %d", max_frames, kPrefetchMaxFrames);
  if (slot_bytes < 1024 || slot_bytes > (int64_t(1) << 40))
    return fail(WV_EINVAL, "wv_prefetch_create: slot_bytes %lld outside 1 KiB .. 2^40", (long long)slot_bytes);
  for (int p = 0; p < c->nplanes; ++p)
    if (wv_sparse_blocks_per_tile(&c->d, p) > kRebuildMaxBlocks)
      return fail(WV_EUNSUPPORTED, "wv_prefetch_create: tiles above 512 samples");
  wv_prefetch* pf = new (std::nothrow) wv_prefetch();
  if (!pf) return fail(WV_ENOMEM, "wv_prefetch_create: allocation failed");
  pf->ctx = c;
  pf->max_frames = max_frames;
  pf->cap = align16((size_t)slot_bytes);
  for (int p = 0; p < c->nplanes; ++p) {
    const int edge = plane_edge(c->d, p);
    pf->kept[p] = kept_table(edge, c->d.levels);
    for (const auto& b : storage_order(edge, c->d.levels)) pf->order[p].push_back((uint16_t)((b.first << 8) | b.second));
  }
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&pf->copy, hipStreamNonBlocking);
  for (int k = 0; e == hipSuccess && k < kPrefetchSlots; ++k) {
    e = hipHostMalloc((void**)&pf->host[k], pf->cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&pf->dev[k], pf->cap);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pf->copied[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pf->consumed[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    const wv_status st = e == hipErrorOutOfMemory ? fail(WV_ENOMEM, "wv_prefetch_create: %s", hipGetErrorString(e))
                                                  : hip_fail(e, "wv_prefetch_create");
    wv_prefetch_destroy(pf);
    return st;
  }
  try {
    pf->worker = std::thread(prepare_thread, pf);
  } catch (...) {
    wv_prefetch_destroy(pf);
    return fail(WV_ENOMEM, "wv_prefetch_create: cannot start the prepare thread");
  }
  *out = pf;
  return WV_OK;
}

extern "C" wv_status wv_prefetch_stage(wv_prefetch* pf, const wv_sparse_plane* frames, int32_t n_frames,
                                       const uint8_t* lc, const uint8_t* mask, int32_t direct, int64_t* bytes) {
  if (!pf || !frames || !mask) return fail(WV_EINVAL, "wv_prefetch_stage: NULL argument");
  if (n_frames < 1 || n_frames > pf->max_frames)
    return fail(WV_EINVAL, "wv_prefetch_stage: n_frames %d outside 1 .. %d", n_frames, pf->max_frames);
  const int k = pf->next_stage;
  {
    std::lock_guard<std::mutex> lock(pf->mu);
    if (pf->slot[k].staged) return fail(WV_EINVAL, "wv_prefetch_stage: two sets are staged and not rebuilt");
  }
  const wv_ctx* c = pf->ctx;
  const int np = c->nplanes, nfp = n_frames * np;
  // layout and record runs of every frame-plane, checked before any work
  StageJob j;
  j.k = k;
  j.direct = direct != 0;
  j.frames.assign(frames, frames + nfp);
  j.runs.resize(nfp);
  j.planes.resize(nfp);
  size_t off = 0;
  for (int t = 0; t < c->n_tiles; ++t) j.n_vis += mask[t] != 0;
  int64_t up = 0;
  for (int i = 0; i < nfp; ++i) {
    const wv_sparse_plane& sp = frames[i];
    const int p = i % np;
    if (!sp.block_end || sp.n_records < 0 || (sp.n_records > 0 && (!sp.values || !sp.index)))
      return fail(WV_EINVAL, "wv_prefetch_stage: frame %d plane %d: missing arrays", i / np, p);
    const wv_status st = tile_runs(&c->d, p, pf->kept[p], sp.block_end, sp.n_records, lc, mask, j.runs[i]);
    if (st != WV_OK) return st;
    int64_t n = 0;
    for (const TileRun& r : j.runs[i]) n += r.end - r.begin;
    StagedPlane& s = j.planes[i];
    const int nb = wv_sparse_blocks_per_tile(&c->d, p);
    s.be_off = off;
    off = align16(off + (size_t)j.n_vis * nb * 4);
    s.idx_off = off;
    off = align16(off + (size_t)n * 2);
    s.val_off = off;
    off = align16(off + (size_t)n);
    s.n = n;
    std::memcpy(s.bounds, sp.bounds, sizeof s.bounds);
    up += (int64_t)j.n_vis * nb * 4 + n * 3;
  }
  if (off > pf->cap)
    return fail(WV_EINVAL, "wv_prefetch_stage: %zu bytes exceed the slot's %zu", off, pf->cap);
  j.bytes = off;
  for (int t = 0; t < c->n_tiles; ++t) {
    if (!mask[t]) continue;
    Item it = {};
    it.tile = (uint16_t)t;
    it.slot = (uint16_t)j.items.size();
    it.lc = (uint8_t)(lc ? lc[t] : c->d.levels);
    j.items.push_back(it);
  }
  {
    std::lock_guard<std::mutex> lock(pf->mu);
    Slot& sl = pf->slot[k];
    sl.staged = true;
    sl.ready = false;
    sl.err = WV_OK;
    sl.n_frames = n_frames;
    sl.items = j.items;
    sl.planes = j.planes;
    pf->jobs.push_back(std::move(j));
  }
  pf->cv.notify_all();
  pf->next_stage = (k + 1) % kPrefetchSlots;
  // bytes uploaded: the whole slot layout when gathered, the block-end
  // tables and the runs themselves when copied run by run
  if (bytes) *bytes = direct ? up : (int64_t)off;
  return WV_OK;
}

extern "C" wv_status wv_prefetch_rebuild(wv_prefetch* pf, void* const* dense, hipStream_t s) {
  if (!pf || !dense) return fail(WV_EINVAL, "wv_prefetch_rebuild: NULL argument");
  const int k = pf->next_rebuild;
  Slot& sl = pf->slot[k];
  {
    std::unique_lock<std::mutex> lock(pf->mu);
    if (!sl.staged) return fail(WV_EINVAL, "wv_prefetch_rebuild: no staged set");
    // the prepare thread has enqueued this set's upload (or failed)
    pf->cv.wait(lock, [&] { return sl.ready; });
    if (sl.err != WV_OK) {
      sl.staged = false;
      pf->next_rebuild = (k + 1) % kPrefetchSlots;
      return fail(sl.err, "%s", sl.msg);
    }
  }
  const wv_ctx* c = pf->ctx;
  const int np = c->nplanes, nfp = sl.n_frames * np;
  for (int i = 0; i < nfp; ++i) {
    if (!dense[i]) return fail(WV_EINVAL, "wv_prefetch_rebuild: dense[%d] is NULL", i);
    if (!aligned16(dense[i])) return fail(WV_EINVAL, "wv_prefetch_rebuild: dense[%d] is not 16-byte aligned", i);
  }
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, pf->copied[k], 0);
  for (int i = 0; e == hipSuccess && i < nfp; ++i) {
    const StagedPlane& sp = sl.planes[i];
    RebuildArgs a;
    memset(&a, 0, sizeof a);
    a.block_end = (const uint32_t*)(pf->dev[k] + sp.be_off);
    a.index = (const uint16_t*)(pf->dev[k] + sp.idx_off);
    a.values = pf->dev[k] + sp.val_off;
    a.n_records = (uint64_t)sp.n;
    a.dense = dense[i];
    a.compact = 1;
    a.p = plane_edge(c->d, i % np);
    a.levels = c->d.levels;
    a.b = block_edge(a.p);
    const std::vector<uint16_t>& order = pf->order[i % np];
    a.nb = (int)order.size();
    std::copy(order.begin(), order.end(), a.order);
    for (int q = 0; q < 2; ++q) {
      const double lo = sp.bounds[2 * q], hi = sp.bounds[2 * q + 1];
      a.lo[q] = (float)lo;
      a.scale[q] = (float)((hi - lo) / 255.0);
    }
    for (size_t i0 = 0; e == hipSuccess && i0 < sl.items.size(); i0 += kArgItems) {
      const int n = (int)std::min<size_t>(kArgItems, sl.items.size() - i0);
      std::copy(sl.items.begin() + i0, sl.items.begin() + i0 + n, a.items);
      a.n_items = n;
      e = launch_rebuild(c->d.wavelet, a, s);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(pf->consumed[k], s);
  if (e != hipSuccess) return hip_fail(e, "wv_prefetch_rebuild");
  {
    std::lock_guard<std::mutex> lock(pf->mu);
    sl.consumed_rec = true;
    sl.staged = false;
  }
  pf->next_rebuild = (k + 1) % kPrefetchSlots;
  return WV_OK;
}

// ---------------------------------------------------------------------------
// File container (Section 3.4)

namespace {

constexpr char kMagic[8] = {'W', 'V', '3', '6', '0', 'F', 'M', 'T'};
constexpr uint32_t kVersion = 1;

struct FileHeader {
  char magic[8];
  uint32_t version;
  int32_t width, height, tile, levels, wavelet, format;
  int32_t n_frames, nplanes;
  uint32_t reserved[5];
};
static_assert(sizeof(FileHeader) == 64, "header layout");

struct FileEntry {              // one frame-plane
  uint64_t offset;              // block-end package; the coefficient package follows
  int64_t n_records;
  float bounds[4];
  uint32_t n_block_ends;
  uint32_t reserved[3];
};
static_assert(sizeof(FileEntry) == 48, "entry layout");

uint64_t pad16(uint64_t v) { return (v + 15) & ~(uint64_t)15; }

// Bytes of one frame-plane's packages: block ends, indices, codes.
uint64_t package_bytes(uint32_t nbe, int64_t n, uint64_t* idx_off, uint64_t* val_off) {
  const uint64_t a = pad16((uint64_t)nbe * 4);
  const uint64_t b = pad16((uint64_t)n * 2);
  *idx_off = a;
  *val_off = a + b;
  return a + b + pad16((uint64_t)n);
}

}  // namespace

struct wv_store {
  wv_desc d;
  int n_frames = 0, nplanes = 0;
  unsigned char* data = nullptr;   // the whole file
  uint64_t size = 0;
  bool pinned = false;
  std::vector<FileEntry> entries;
};

extern "C" wv_status wv_store_write(const char* path, const wv_desc* d, int32_t n_frames,
                                    const wv_sparse_plane* frames) {
  if (!path || !d || !frames || n_frames < 1) return fail(WV_EINVAL, "wv_store_write: bad argument");
  const wv_status st = check_desc(d);
  if (st != WV_OK) return st;
  const int np = d->format == WV_YUV420 ? 3 : 1;
  const int n_tiles = (d->width / d->tile) * (d->height / d->tile);
  const int nfp = n_frames * np;
  std::vector<FileEntry> entries(nfp);
  uint64_t off = pad16(sizeof(FileHeader) + (uint64_t)nfp * sizeof(FileEntry));
  for (int i = 0; i < nfp; ++i) {
    const wv_sparse_plane& sp = frames[i];
    if (!sp.block_end || sp.n_records < 0 || (sp.n_records > 0 && (!sp.values || !sp.index)))
      return fail(WV_EINVAL, "wv_store_write: frame %d plane %d: missing arrays", i / np, i % np);
    FileEntry& e = entries[i];
    std::memset(&e, 0, sizeof e);
    e.offset = off;
    e.n_records = sp.n_records;
    std::memcpy(e.bounds, sp.bounds, sizeof e.bounds);
    e.n_block_ends = (uint32_t)(n_tiles * wv_sparse_blocks_per_tile(d, i % np));
    uint64_t io, vo;
    off += package_bytes(e.n_block_ends, e.n_records, &io, &vo);
  }
  FileHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kMagic, sizeof kMagic);
  h.version = kVersion;
  h.width = d->width;
  h.height = d->height;
  h.tile = d->tile;
  h.levels = d->levels;
  h.wavelet = d->wavelet;
  h.format = d->format;
  h.n_frames = n_frames;
  h.nplanes = np;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(WV_EDEVICE, "wv_store_write: cannot open %s", path);
  static const unsigned char zeros[16] = {};
  auto put = [&](const void* p, uint64_t n) { return n == 0 || std::fwrite(p, 1, n, f) == n; };
  auto pad_to = [&](uint64_t at, uint64_t want) { return put(zeros, want - at); };
  bool ok = put(&h, sizeof h) && put(entries.data(), (uint64_t)nfp * sizeof(FileEntry));
  uint64_t at = sizeof h + (uint64_t)nfp * sizeof(FileEntry);
  ok = ok && pad_to(at, pad16(at));
  at = pad16(at);
  for (int i = 0; ok && i < nfp; ++i) {
    const wv_sparse_plane& sp = frames[i];
    const FileEntry& e = entries[i];
    uint64_t io, vo;
    const uint64_t total = package_bytes(e.n_block_ends, e.n_records, &io, &vo);
    ok = put(sp.block_end, (uint64_t)e.n_block_ends * 4) && pad_to((uint64_t)e.n_block_ends * 4, io) &&
         put(sp.index, (uint64_t)e.n_records * 2) && pad_to(io + (uint64_t)e.n_records * 2, vo) &&
         put(sp.values, (uint64_t)e.n_records) && pad_to(vo + (uint64_t)e.n_records, total);
    at += total;
  }
  if (std::fclose(f) != 0) ok = false;
  if (!ok) return fail(WV_EDEVICE, "wv_store_write: write to %s failed", path);
  return WV_OK;
}

extern "C" wv_status wv_store_close(wv_store* s) {
  if (!s) return WV_OK;
  if (s->data) {
    if (s->pinned) hipHostFree(s->data);
    else std::free(s->data);
  }
  delete s;
  return WV_OK;
}

extern "C" wv_status wv_store_open(const char* path, int32_t pinned, wv_store** out) {
  if (!path || !out) return fail(WV_EINVAL, "wv_store_open: bad argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(WV_EINVAL, "wv_store_open: cannot open %s", path);
  std::fseek(f, 0, SEEK_END);
  const long len = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  if (len < (long)sizeof(FileHeader)) {
    std::fclose(f);
    return fail(WV_EINVAL, "wv_store_open: %s is too short for a header", path);
  }
  wv_store* s = new (std::nothrow) wv_store();
  if (!s) {
    std::fclose(f);
    return fail(WV_ENOMEM, "wv_store_open: allocation failed");
  }
  s->size = (uint64_t)len;
  s->pinned = pinned != 0;
  if (s->pinned) {
    if (hipHostMalloc((void**)&s->data, s->size, hipHostMallocDefault) != hipSuccess) s->data = nullptr;
  } else {
    s->data = (unsigned char*)std::malloc(s->size);
  }
  if (!s->data) {
    std::fclose(f);
    wv_store_close(s);
    return fail(WV_ENOMEM, "wv_store_open: %llu bytes", (unsigned long long)len);
  }
  const bool read_ok = std::fread(s->data, 1, s->size, f) == s->size;
  std::fclose(f);
  if (!read_ok) {
    wv_store_close(s);
    return fail(WV_EDEVICE, "wv_store_open: read of %s failed", path);
  }
  FileHeader h;
  std::memcpy(&h, s->data, sizeof h);
  wv_desc d = {};
  d.width = h.width;
  d.height = h.height;
  d.tile = h.tile;
  d.levels = h.levels;
  d.wavelet = h.wavelet;
  d.format = h.format;
  const int np = d.format == WV_YUV420 ? 3 : 1;
  if (std::memcmp(h.magic, kMagic, sizeof kMagic) != 0 || h.version != kVersion || check_desc(&d) != WV_OK ||
      h.n_frames < 1 || h.nplanes != np ||
      sizeof h + (uint64_t)h.n_frames * np * sizeof(FileEntry) > s->size) {
    wv_store_close(s);
    return fail(WV_EINVAL, "wv_store_open: %s is not a valid file of this format", path);
  }
  s->d = d;
  s->n_frames = h.n_frames;
  s->nplanes = np;
  s->entries.resize((size_t)h.n_frames * np);
  std::memcpy(s->entries.data(), s->data + sizeof h, s->entries.size() * sizeof(FileEntry));
  const int n_tiles = (d.width / d.tile) * (d.height / d.tile);
  for (size_t i = 0; i < s->entries.size(); ++i) {
    const FileEntry& e = s->entries[i];
    uint64_t io, vo;
    const uint64_t nbe = (uint64_t)n_tiles * wv_sparse_blocks_per_tile(&d, (int)(i % np));
    if (e.n_records < 0 || e.n_block_ends != nbe || e.offset % 16 ||
        e.offset + package_bytes(e.n_block_ends, e.n_records, &io, &vo) > s->size) {
      wv_store_close(s);
      return fail(WV_EINVAL, "wv_store_open: %s: entry %zu is inconsistent", path, i);
    }
  }
  *out = s;
  return WV_OK;
}

extern "C" wv_status wv_store_info(const wv_store* s, wv_desc* d, int32_t* n_frames) {
  if (!s || !d || !n_frames) return fail(WV_EINVAL, "wv_store_info: bad argument");
  *d = s->d;
  *n_frames = s->n_frames;
  return WV_OK;
}

extern "C" wv_status wv_store_frame(const wv_store* s, int32_t frame, wv_sparse_plane* planes) {
  if (!s || !planes) return fail(WV_EINVAL, "wv_store_frame: bad argument");
  if (frame < 0 || frame >= s->n_frames)
    return fail(WV_EINVAL, "wv_store_frame: frame %d outside 0 .. %d", frame, s->n_frames - 1);
  for (int p = 0; p < s->nplanes; ++p) {
    const FileEntry& e = s->entries[(size_t)frame * s->nplanes + p];
    uint64_t io, vo;
    package_bytes(e.n_block_ends, e.n_records, &io, &vo);
    wv_sparse_plane& sp = planes[p];
    sp.block_end = (const uint32_t*)(s->data + e.offset);
    sp.index = (const uint16_t*)(s->data + e.offset + io);
    sp.values = s->data + e.offset + vo;
    sp.n_records = e.n_records;
    std::memcpy(sp.bounds, e.bounds, sizeof sp.bounds);
  }
  return WV_OK;
}
