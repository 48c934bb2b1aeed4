// Serving loop: many head-tracked streams decoded with continuous batching.
//
// Each stream plays a GOP source (device-resident coefficient planes) and
// requests frames at its own times and head poses.  Streams are admitted
// into slots -- device-resident reference planes plus an output buffer --
// whose number is set by an HBM budget; a finished stream frees its slot for
// the next one.  The loop never waits for a batch to finish before accepting
// work: at every turn it takes the requests that have arrived, builds the
// viewport jobs of all of them (tiles that entered a viewport since their
// last reconstruction are replayed first, in earlier rounds), and launches
// each round as ONE persistent kernel replayed from a captured hipGraph
// whose work table is rewritten per round.  Up to two turns are in flight;
// HIP stream order keeps every stream's frames in sequence.  Completion
// times come from HIP events, latencies are completion minus arrival.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "wv_ctx.h"
#include "wv_geom.h"

using namespace wv;
using namespace wvp;

namespace {

constexpr int kSrvJobs = 256;          // jobs per round (one per active stream)
constexpr int kSrvItems = 16384;       // visible tiles per round
constexpr size_t kHdr = 256;           // header: unit count at offset 0
constexpr size_t kSrvTab = kHdr + kSrvJobs * sizeof(Job) + kSrvItems * sizeof(Item);

// Per-tile sample directions (each tile with its own eye) do not depend on
// the head pose, so they are computed once; a pose then costs dot products.
// The decisions are those of wv_viewport_mask / wv_foveation_levels: the
// same expressions on the same doubles.  A tile whose centre lies further
// from the gaze than the frustum's half-diagonal plus the tile's own angular
// radius has no sample inside and is skipped without testing its samples.
struct DirTable {
  int samples = 0, n = 0;
  std::vector<double> dir;      // [tile][samples^2][3]
  std::vector<double> centre;   // [tile][3]
  std::vector<double> radius;   // [tile] max angle (rad) from centre to a sample
  std::vector<int> eye;         // [tile]
};

void build_dirs(DirTable& t, const wv_desc& d, int samples) {
  const int ntx = d.width / d.tile, nty = d.height / d.tile, ss = samples * samples;
  const double eye_h = d.height / 2.0;
  t.samples = samples;
  t.n = ntx * nty;
  t.dir.resize((size_t)t.n * ss * 3);
  t.centre.resize((size_t)t.n * 3);
  t.radius.resize(t.n);
  t.eye.resize(t.n);
  for (int ty = 0; ty < nty; ++ty)
    for (int tx = 0; tx < ntx; ++tx) {
      const int id = ty * ntx + tx;
      t.eye[id] = wvg::tile_eye(ty, d.tile, eye_h);
      double* c = &t.centre[id * 3];
      wvg::centre_direction(tx, ty, d.tile, (double)d.width, eye_h, c);
      double rmax = 0.0;
      for (int i = 0; i < samples; ++i)
        for (int j = 0; j < samples; ++j) {
          double* p = &t.dir[((size_t)id * ss + i * samples + j) * 3];
          wvg::sample_direction(tx, ty, i, j, d.tile, samples, (double)d.width, eye_h, p);
          rmax = std::fmax(rmax, std::acos(std::fmax(-1.0, std::fmin(1.0, wvg::dot(p, c)))));
        }
      t.radius[id] = rmax + 1e-9;
    }
}

// Mask and level counts of one pose.
void select_tiles(const DirTable& t, int levels, const wv_view_class& v, double yaw, double pitch,
                  uint8_t* mask, uint8_t* lc) {
  const wvg::Camera c = wvg::camera(yaw, pitch);
  const double th = std::tan(v.fov_h * (M_PI / 360.0)), tv = std::tan(v.fov_v * (M_PI / 360.0));
  const double half_diag = std::atan(std::sqrt(th * th + tv * tv)) + 1e-9;
  const int ss = t.samples * t.samples;
  for (int id = 0; id < t.n; ++id) {
    const double* cc = &t.centre[id * 3];
    const double ecc = wvg::eccentricity(cc, c);
    uint8_t hit = 0;
    if (t.eye[id] < v.eyes && ecc * (M_PI / 180.0) - t.radius[id] <= half_diag) {
      const double* p = &t.dir[(size_t)id * ss * 3];
      for (int k = 0; k < ss && !hit; ++k, p += 3)
        if (wvg::in_frustum(p, c, th, tv)) hit = 1;
    }
    mask[id] = hit;
    lc[id] = (uint8_t)(v.foveate ? wvg::foveated_levels(levels, ecc, v.inner, v.outer) : levels);
  }
}

struct Source {
  std::vector<wv_frame> frames;   // one GOP: frame 0 intra, the rest residual
};

struct StreamRec {
  wv_stream_desc d;
  std::vector<double> arrival, yaw, pitch;
  std::vector<void*> outs;        // per frame, or empty (slot buffer)
  int slot = -1;
  int next = 0;                   // next frame to enqueue
  int completed = 0;              // frames whose turn has completed
  int req_base = 0;               // global index of frame 0
  bool admitted = false, finished = false;
};

struct Slot {
  void* ref[3] = {};
  void* out = nullptr;
  std::vector<int32_t> stamp;     // last reconstructed frame per tile
  int stream = -1;
};

// Requests enqueued together and the event that marks their completion.
struct Turn {
  hipEvent_t done = nullptr;
  std::vector<int> reqs, streams;
  bool busy = false;
};

// Jobs of one launch: at most one per stream.
struct Round {
  std::vector<Job> jobs;
  std::vector<Item> items;
};

}  // namespace

struct wv_server {
  wv_ctx* ctx = nullptr;
  wv_desc d;
  int max_vis = 0;
  int n_slots = 0;
  int variant = -1;                // persistent fused variant replayed by the graphs
  int bpt = 0;                     // work units per tile
  std::vector<Slot> slots;
  std::vector<Source> sources;
  std::vector<StreamRec> streams;
  DirTable dirs;
  // Double-buffered work tables (pinned host + device) and the graphs that
  // copy one to the device and run the persistent kernel over it.
  unsigned char* hst[2] = {};
  unsigned char* dev[2] = {};
  hipGraph_t graph[2] = {};
  hipGraphExec_t gexec[2] = {};
  hipEvent_t tab_free[2] = {};
  int next_tab = 0;
  hipStream_t cap = nullptr;
};

namespace {

wv_status build_graphs(wv_server* s) {
  const Variant* var = fused_variant(s->d.wavelet, s->d.format, s->variant);
  for (int k = 0; k < 2; ++k) {
    WorkArgs a;
    memset(&a, 0, sizeof a);
    fill_geometry(s->ctx, var, a);
    a.total_dev = (const int32_t*)s->dev[k];
    a.jobs_dev = (const Job*)(s->dev[k] + kHdr);
    a.items_dev = (const Item*)(s->dev[k] + kHdr + kSrvJobs * sizeof(Job));
    a.total = s->ctx->n_cu * var->groups_per_cu;   // sizes the persistent grid only
    hipError_t e = hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "server graph capture");
    hipError_t el = hipMemcpyAsync(s->dev[k], s->hst[k], kSrvTab, hipMemcpyHostToDevice, s->cap);
    if (el == hipSuccess) el = launch_fused(s->d.wavelet, s->d.format, s->variant, a, s->ctx->n_cu, s->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s->cap, &g);
    if (g) s->graph[k] = g;
    if (el != hipSuccess) return hip_fail(el, "server graph capture");
    if (e != hipSuccess) return hip_fail(e, "server graph capture");
    e = hipGraphInstantiate(&s->gexec[k], g, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "server graph instantiate");
  }
  return WV_OK;
}

// Copy a round into the next work table and replay that table's graph; a
// round above the table's capacity goes out in several launches.
wv_status launch_round(wv_server* s, const Round& rd, hipStream_t stream, int64_t* launches) {
  for (size_t i0 = 0; i0 < rd.items.size(); i0 += kSrvItems) {
    const size_t n = std::min<size_t>(kSrvItems, rd.items.size() - i0);
    const int k = s->next_tab;
    s->next_tab ^= 1;
    hipError_t e = hipEventSynchronize(s->tab_free[k]);   // the launch that last read table k
    if (e != hipSuccess) return hip_fail(e, "server table wait");
    unsigned char* h = s->hst[k];
    *(int32_t*)h = (int32_t)(n * s->bpt);
    memcpy(h + kHdr, rd.jobs.data(), rd.jobs.size() * sizeof(Job));
    memcpy(h + kHdr + kSrvJobs * sizeof(Job), rd.items.data() + i0, n * sizeof(Item));
    e = hipGraphLaunch(s->gexec[k], stream);
    if (e == hipSuccess) e = hipEventRecord(s->tab_free[k], stream);
    if (e != hipSuccess) return hip_fail(e, "server graph launch");
    ++*launches;
  }
  return WV_OK;
}

}  // namespace

extern "C" wv_status wv_server_destroy(wv_server* s) {
  if (!s) return WV_OK;
  if (s->cap) (void)hipStreamSynchronize(s->cap);
  for (int k = 0; k < 2; ++k)
    if (s->tab_free[k]) (void)hipEventSynchronize(s->tab_free[k]);
  for (Slot& sl : s->slots) {
    for (void* p : sl.ref)
      if (p) (void)hipFree(p);
    if (sl.out) (void)hipFree(sl.out);
  }
  for (int k = 0; k < 2; ++k) {
    if (s->gexec[k]) (void)hipGraphExecDestroy(s->gexec[k]);
    if (s->graph[k]) (void)hipGraphDestroy(s->graph[k]);
    if (s->hst[k]) (void)hipHostFree(s->hst[k]);
    if (s->dev[k]) (void)hipFree(s->dev[k]);
    if (s->tab_free[k]) (void)hipEventDestroy(s->tab_free[k]);
  }
  if (s->cap) (void)hipStreamDestroy(s->cap);
  if (s->ctx) wv_destroy(s->ctx);
  delete s;
  return WV_OK;
}

extern "C" wv_status wv_server_create(wv_server** out, const wv_desc* desc, int32_t max_active,
                                      int64_t hbm_budget, int32_t max_visible) {
  if (!out) return fail(WV_EINVAL, "wv_server_create: out is NULL");
  *out = nullptr;
  if (!desc || max_active < 1 || max_active > kSrvJobs || hbm_budget <= 0 || max_visible < 1)
    return fail(WV_EINVAL, "wv_server_create: bad argument (max_active 1..%d)", kSrvJobs);
  wv_server* s = new (std::nothrow) wv_server();
  if (!s) return fail(WV_ENOMEM, "server allocation");
  wv_status st = wv_create(&s->ctx, desc);
  if (st != WV_OK) {
    delete s;
    return st;
  }
  s->d = *desc;
  const int n_tiles = s->ctx->n_tiles, np = s->ctx->nplanes;
  s->max_vis = std::min(max_visible, n_tiles);
  for (int v = 0; v < fused_variant_count(desc->wavelet, desc->format); ++v) {
    const Variant* var = fused_variant(desc->wavelet, desc->format, v);
    if (var->persistent && variant_fits(*desc, var)) {
      s->variant = v;
      s->bpt = (desc->tile / var->bw) * (desc->tile / var->bh);
      break;
    }
  }
  if (s->variant < 0) {
    wv_server_destroy(s);
    return fail(WV_EUNSUPPORTED, "no persistent fused variant fits this geometry");
  }
  // one slot: the reference planes of every tile plus one frame of output
  const size_t T2 = (size_t)desc->tile * desc->tile, sb = sample_bytes(*desc);
  size_t ref_bytes = 0;
  for (int p = 0; p < np; ++p) ref_bytes += (size_t)n_tiles * plane_edge(*desc, p) * plane_edge(*desc, p) * sb;
  const size_t out_bytes = (size_t)s->max_vis * np * T2 * sb;
  const int64_t slot_bytes = (int64_t)(ref_bytes + out_bytes);
  s->n_slots = (int)std::min<int64_t>(max_active, hbm_budget / slot_bytes);
  if (s->n_slots < 1) {
    wv_server_destroy(s);
    return fail(WV_ENOMEM, "HBM budget %lld below one stream slot (%lld bytes)", (long long)hbm_budget,
                (long long)slot_bytes);
  }
  s->slots.resize(s->n_slots);
  hipError_t e = hipSuccess;
  for (Slot& sl : s->slots) {
    for (int p = 0; p < np && e == hipSuccess; ++p) {
      const size_t P = plane_edge(*desc, p);
      e = hipMalloc(&sl.ref[p], (size_t)n_tiles * P * P * sb);
    }
    if (e == hipSuccess) e = hipMalloc(&sl.out, out_bytes);
    if (e != hipSuccess) break;
    sl.stamp.assign(n_tiles, -1);
  }
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipHostMalloc((void**)&s->hst[k], kSrvTab, hipHostMallocDefault);
    if (e == hipSuccess) memset(s->hst[k], 0, kSrvTab);
    if (e == hipSuccess) e = hipMalloc((void**)&s->dev[k], kSrvTab);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->tab_free[k], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    wv_server_destroy(s);
    return e == hipErrorOutOfMemory ? fail(WV_ENOMEM, "server slots: %s", hipGetErrorString(e))
                                    : hip_fail(e, "wv_server_create");
  }
  if ((st = build_graphs(s)) != WV_OK) {
    wv_server_destroy(s);
    return st;
  }
  build_dirs(s->dirs, *desc, 16);
  *out = s;
  return WV_OK;
}

extern "C" int32_t wv_server_slots(const wv_server* s) { return s ? s->n_slots : 0; }

extern "C" wv_status wv_server_add_source(wv_server* s, int32_t gop_len, const wv_frame* frames) {
  if (!s || gop_len < 1 || !frames) return fail(WV_EINVAL, "wv_server_add_source: bad argument");
  Source src;
  for (int i = 0; i < gop_len; ++i) {
    const wv_frame& f = frames[i];
    for (int p = 0; p < s->ctx->nplanes; ++p)
      if (!f.planes[p] || !aligned16(f.planes[p]))
        return fail(WV_EINVAL, "source frame %d plane %d: NULL or not 16-byte aligned", i, p);
    if ((i == 0) != (f.is_intra != 0))
      return fail(WV_EINVAL, "source frame %d: frame 0 must be the only intra frame", i);
    if (s->d.wavelet == WV_W53 && (f.qstep < 1 || f.qstep > 65535))
      return fail(WV_EINVAL, "source frame %d: qstep %d out of range", i, f.qstep);
    src.frames.push_back(f);
  }
  s->sources.push_back(src);
  return WV_OK;
}

extern "C" wv_status wv_server_add_stream(wv_server* s, const wv_stream_desc* sd) {
  if (!s || !sd || sd->n_frames < 1 || !sd->arrival || !sd->yaw || !sd->pitch)
    return fail(WV_EINVAL, "wv_server_add_stream: bad argument");
  if (sd->source < 0 || sd->source >= (int)s->sources.size())
    return fail(WV_EINVAL, "stream source %d out of range", sd->source);
  const wv_view_class& v = sd->view;
  if (!(v.fov_h > 0 && v.fov_h < 180 && v.fov_v > 0 && v.fov_v < 180) || (v.eyes != 1 && v.eyes != 2) ||
      (v.foveate && !(v.inner >= 0 && v.outer >= v.inner)))
    return fail(WV_EINVAL, "stream view class out of range");
  StreamRec r;
  r.d = *sd;
  r.arrival.assign(sd->arrival, sd->arrival + sd->n_frames);
  r.yaw.assign(sd->yaw, sd->yaw + sd->n_frames);
  r.pitch.assign(sd->pitch, sd->pitch + sd->n_frames);
  for (int i = 0; i < sd->n_frames; ++i)
    if (!(r.arrival[i] >= (i ? r.arrival[i - 1] : 0.0)))
      return fail(WV_EINVAL, "stream arrival times must be >= 0 and not decrease");
  if (sd->out_frames) {
    r.outs.assign(sd->out_frames, sd->out_frames + sd->n_frames);
    for (void* p : r.outs)
      if (!p || !aligned16(p)) return fail(WV_EINVAL, "stream out_frames entry NULL or not 16-byte aligned");
  }
  r.d.arrival = r.d.yaw = r.d.pitch = nullptr;
  r.d.out_frames = nullptr;
  s->streams.push_back(std::move(r));
  return WV_OK;
}

extern "C" wv_status wv_server_clear_streams(wv_server* s) {
  if (!s) return fail(WV_EINVAL, "wv_server_clear_streams: NULL server");
  s->streams.clear();
  return WV_OK;
}

extern "C" wv_status wv_server_run(wv_server* s, double time_scale, double* latency_ms,
                                   wv_server_stats* stats, hipStream_t stream) {
  if (!s || !(time_scale >= 0)) return fail(WV_EINVAL, "wv_server_run: bad argument");
  const int n_tiles = s->ctx->n_tiles, levels = s->d.levels;
  const double T2 = (double)s->d.tile * s->d.tile;
  int total_req = 0;
  for (StreamRec& r : s->streams) {
    r.req_base = total_req;
    total_req += r.d.n_frames;
    r.slot = -1;
    r.next = r.completed = 0;
    r.admitted = r.finished = false;
  }
  for (Slot& sl : s->slots) sl.stream = -1;
  std::vector<double> lat(total_req, -1.0), arr_ms(total_req, 0.0);
  for (const StreamRec& r : s->streams)
    for (int i = 0; i < r.d.n_frames; ++i) arr_ms[r.req_base + i] = r.arrival[i] * time_scale * 1e3;
  wv_server_stats st;
  memset(&st, 0, sizeof st);
  st.requests = total_req;

  hipEvent_t t0 = nullptr;
  Turn turns[2];
  hipError_t e = hipEventCreate(&t0);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreate(&turns[k].done);
  // start the clocks together: GPU times are read against t0
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e == hipSuccess) e = hipEventRecord(t0, stream);
  if (e == hipSuccess) e = hipEventSynchronize(t0);
  const auto wall0 = std::chrono::steady_clock::now();
  wv_status result = e == hipSuccess ? WV_OK : hip_fail(e, "server start");
  auto wall_s = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count(); };

  auto retire = [&](Turn& t) -> wv_status {
    float ms = 0.f;
    const hipError_t ee = hipEventElapsedTime(&ms, t0, t.done);
    if (ee != hipSuccess) return hip_fail(ee, "server completion time");
    st.gpu_ms = std::max(st.gpu_ms, (double)ms);
    for (size_t i = 0; i < t.reqs.size(); ++i) {
      lat[t.reqs[i]] = (double)ms - arr_ms[t.reqs[i]];
      StreamRec& r = s->streams[t.streams[i]];
      if (++r.completed == r.d.n_frames) {
        r.finished = true;
        s->slots[r.slot].stream = -1;   // later turns of this slot are already ordered after it
      }
    }
    t.reqs.clear();
    t.streams.clear();
    t.busy = false;
    return WV_OK;
  };

  std::vector<uint8_t> mask(n_tiles), lc(n_tiles), maskf(n_tiles), lcf(n_tiles);
  std::vector<int> from(n_tiles);
  std::vector<Round> rounds;
  size_t next_pending = 0;
  int finished = 0, cur = 0;
  while (result == WV_OK) {
    // retire completed turns without blocking
    for (Turn& t : turns)
      if (result == WV_OK && t.busy && hipEventQuery(t.done) == hipSuccess) result = retire(t);
    if (result != WV_OK) break;
    finished = 0;
    int active = 0;
    for (const StreamRec& r : s->streams) {
      finished += r.finished;
      active += r.admitted && !r.finished;
    }
    if (finished == (int)s->streams.size()) break;
    // admission: free slots go to waiting streams in the order they were added
    for (int i = 0; i < s->n_slots && next_pending < s->streams.size(); ++i) {
      Slot& sl = s->slots[i];
      if (sl.stream >= 0) continue;
      StreamRec& r = s->streams[next_pending];
      r.slot = i;
      r.admitted = true;
      sl.stream = (int)next_pending++;
      std::fill(sl.stamp.begin(), sl.stamp.end(), -1);
      ++st.admitted;
      ++active;
    }
    st.max_active = std::max<int64_t>(st.max_active, active);
    Turn& tn = turns[cur];
    if (tn.busy) {   // two turns in flight: wait for the older one
      e = hipEventSynchronize(tn.done);
      result = e == hipSuccess ? retire(tn) : hip_fail(e, "server turn wait");
      continue;
    }
    // the arrived next frame of every admitted stream
    const double now = time_scale > 0 ? wall_s() : 0.0;
    double next_arrival = 1e300;
    struct Req {
      int stream, frame, start;
    };
    std::vector<Req> reqs;
    int max_depth = 0;
    for (int si = 0; si < (int)s->streams.size(); ++si) {
      StreamRec& r = s->streams[si];
      if (!r.admitted || r.finished || r.next >= r.d.n_frames) continue;
      const double at = r.arrival[r.next] * time_scale;
      if (at > now) {
        next_arrival = std::min(next_arrival, at);
        continue;
      }
      const Slot& sl = s->slots[r.slot];
      const int gl = (int)s->sources[r.d.source].frames.size();
      const int t = r.next, g0 = t - t % gl;
      select_tiles(s->dirs, levels, r.d.view, r.yaw[t], r.pitch[t], mask.data(), lc.data());
      int start = t;
      for (int x = 0; x < n_tiles; ++x)
        if (mask[x]) start = std::min(start, sl.stamp[x] >= g0 ? sl.stamp[x] + 1 : g0);
      reqs.push_back({si, t, start});
      max_depth = std::max(max_depth, t - start);
    }
    if (reqs.empty()) {
      if (!turns[0].busy && !turns[1].busy && next_arrival < 1e299) {
        const double wait = next_arrival - wall_s();
        if (wait > 1e-3) std::this_thread::sleep_for(std::chrono::duration<double>(wait - 5e-4));
      } else {
        std::this_thread::yield();
      }
      continue;
    }
    // rounds aligned at the end: every request's own frame is in the last one
    rounds.assign(max_depth + 1, Round());
    for (const Req& q : reqs) {
      StreamRec& r = s->streams[q.stream];
      Slot& sl = s->slots[r.slot];
      const Source& src = s->sources[r.d.source];
      const int gl = (int)src.frames.size(), t = q.frame, g0 = t - t % gl;
      select_tiles(s->dirs, levels, r.d.view, r.yaw[t], r.pitch[t], mask.data(), lc.data());
      int n_vis = 0;
      for (int x = 0; x < n_tiles; ++x)
        if (mask[x]) {
          from[x] = sl.stamp[x] >= g0 ? sl.stamp[x] + 1 : g0;
          ++n_vis;
        }
      if (n_vis > s->max_vis) {
        result = fail(WV_EUNSUPPORTED, "stream %d frame %d: %d visible tiles, above max_visible %d", q.stream,
                      t, n_vis, s->max_vis);
        break;
      }
      wv_ref ref{{sl.ref[0], sl.ref[1], sl.ref[2]}, sl.stamp.data()};
      // replays: frame f of every visible tile that lacks it, at the level
      // counts of frame f's own pose
      for (int f = q.start; f < t; ++f) {
        select_tiles(s->dirs, levels, r.d.view, r.yaw[f], r.pitch[f], maskf.data(), lcf.data());
        Round& rd = rounds[max_depth - (t - f)];
        wv_frame fr = src.frames[f % gl];
        fr.frame_index = f;
        const int ji = (int)rd.jobs.size();
        rd.jobs.push_back(make_job(s->ctx, &fr, &ref, nullptr));
        for (int x = 0; x < n_tiles; ++x)
          if (mask[x] && from[x] <= f) {
            rd.items.push_back(Item{(uint16_t)x, 0, (uint8_t)ji, lcf[x], 0});
            ++st.catchup_tiles;
          }
      }
      // the requested frame
      Round& rd = rounds[max_depth];
      wv_frame fr = src.frames[t % gl];
      fr.frame_index = t;
      const int ji = (int)rd.jobs.size();
      rd.jobs.push_back(make_job(s->ctx, &fr, &ref, r.outs.empty() ? sl.out : r.outs[t]));
      uint16_t slot_i = 0;
      for (int x = 0; x < n_tiles; ++x)
        if (mask[x]) {
          rd.items.push_back(Item{(uint16_t)x, slot_i++, (uint8_t)ji, lc[x], 0});
          sl.stamp[x] = t;
        }
      st.tiles_decoded += slot_i;
      st.mpix += slot_i * T2 / 1e6;
      ++st.frames_decoded;
      tn.reqs.push_back(r.req_base + t);
      tn.streams.push_back(q.stream);
      ++r.next;
    }
    for (const Round& rd : rounds)
      if (result == WV_OK && !rd.items.empty()) result = launch_round(s, rd, stream, &st.launches);
    if (result != WV_OK) break;
    e = hipEventRecord(tn.done, stream);
    if (e != hipSuccess) {
      result = hip_fail(e, "server turn event");
      break;
    }
    tn.busy = true;
    ++st.turns;
    cur ^= 1;
  }
  // drain whatever is in flight, also after an error
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess && result == WV_OK) result = hip_fail(e, "server drain");
  for (Turn& t : turns)
    if (t.busy && result == WV_OK) result = retire(t);
  st.wall_s = wall_s();
  std::vector<double> sorted;
  for (double v : lat)
    if (v >= 0) sorted.push_back(v);
  std::sort(sorted.begin(), sorted.end());
  if (!sorted.empty()) {
    auto pct = [&](double q) { return sorted[(size_t)std::ceil(q * sorted.size()) - 1]; };
    st.p50_ms = pct(0.50);
    st.p99_ms = pct(0.99);
    st.max_ms = sorted.back();
    double sum = 0;
    for (double v : sorted) sum += v;
    st.mean_ms = sum / sorted.size();
  }
  if (latency_ms) std::copy(lat.begin(), lat.end(), latency_ms);
  if (stats) *stats = st;
  (void)hipEventDestroy(t0);
  for (Turn& t : turns)
    if (t.done) (void)hipEventDestroy(t.done);
  return result;
}
