// Host side of libwv: argument validation, reference stamps, work lists,
// kernel launches, the fused-variant tuner and the encoder entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "wv_ctx.h"

using namespace wv;

namespace wvp {

thread_local char g_err[512] = "";

wv_status fail(wv_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

wv_status hip_fail(hipError_t e, const char* what) {
  return fail(WV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool variant_fits(const wv_desc& d, const Variant* v) {
  if (v && v->format >= 0 && v->format != d.format) return false;
  if (v && v->wavelet >= 0 && v->wavelet != d.wavelet) return false;
  if (v && v->kind == 2)   // row strips: compiled for one tile edge and level count
    return d.tile == v->bw && d.levels == v->levels;
  const int min_edge = d.format == WV_YUV420 ? d.tile / 2 : d.tile;
  if (v && !v->general && (min_edge >> (d.levels - 1)) < 16) return false;
  if (v && v->levels != 0 && v->levels != d.levels) return false;
  return v && v->bw <= d.tile && v->bh <= d.tile && d.tile % v->bw == 0 && d.tile % v->bh == 0 &&
         (d.format == WV_GRAY8 || (v->bw / 2 >= 2 && (v->bw / 2) % 2 == 0 && v->bh / 2 >= 2 &&
                                   (v->bh / 2) % 2 == 0));
}

}  // namespace wvp

using namespace wvp;

wv_status wvp::check_desc(const wv_desc* d) {
  if (!d) return fail(WV_EINVAL, "desc is NULL");
  if (d->wavelet != WV_W53 && d->wavelet != WV_W97) return fail(WV_EINVAL, "bad wavelet %d", d->wavelet);
  if (d->format != WV_GRAY8 && d->format != WV_YUV420) return fail(WV_EINVAL, "bad format %d", d->format);
  if (!is_pow2(d->tile) || d->tile < 8 || d->tile > 512)
    return fail(WV_EINVAL, "tile must be a power of two in 8..512 (got %d)", d->tile);
  if (d->width <= 0 || d->height <= 0 || d->width % d->tile || d->height % d->tile)
    return fail(WV_EINVAL, "width/height must be positive multiples of tile");
  const int pc = d->format == WV_YUV420 ? d->tile / 2 : d->tile;
  if (d->levels < 1 || (pc >> d->levels) < 1)
    return fail(WV_EINVAL, "levels must be >= 1 and leave at least one approximation sample");
  const long n = (long)(d->width / d->tile) * (d->height / d->tile);
  if (n > 65535) return fail(WV_EINVAL, "at most 65535 tiles per frame");
  return WV_OK;
}

extern "C" {

const char* wv_strerror(wv_status s) {
  switch (s) {
    case WV_OK: return "ok";
    case WV_EINVAL: return "invalid argument";
    case WV_ESTALE: return "stale reference: a residual frame's tile lacks the previous frame";
    case WV_ENOMEM: return "out of memory";
    case WV_EDEVICE: return "HIP device error";
    case WV_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

const char* wv_last_error(void) { return g_err; }

wv_status wv_create(wv_ctx** out, const wv_desc* desc) {
  g_err[0] = 0;
  if (!out) return fail(WV_EINVAL, "ctx out-pointer is NULL");
  *out = nullptr;
  wv_status st = check_desc(desc);
  if (st != WV_OK) return st;
  wv_ctx* c = new (std::nothrow) wv_ctx();
  if (!c) return fail(WV_ENOMEM, "context allocation failed");
  c->d = *desc;
  c->n_tiles = (desc->width / desc->tile) * (desc->height / desc->tile);
  c->nplanes = desc->format == WV_YUV420 ? 3 : 1;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e == hipSuccess) e = hipMalloc((void**)&c->counter, 2 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(c->counter, 0, 2 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->tab_host, kTableSlots * kTableBytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void**)&c->tab_dev, kTableSlots * kTableBytes);
  for (int i = 0; e == hipSuccess && i < kTableSlots; ++i)
    e = hipEventCreateWithFlags(&c->tab_done[i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    st = e == hipErrorOutOfMemory ? fail(WV_ENOMEM, "wv_create: %s", hipGetErrorString(e))
                                  : hip_fail(e, "wv_create");
    wv_destroy(c);
    return st;
  }
  // default variant: the first that fits the tile geometry
  c->variant = -1;
  for (int v = 0; v < fused_variant_count(desc->wavelet, desc->format); ++v)
    if (variant_fits(c->d, fused_variant(desc->wavelet, desc->format, v))) { c->variant = v; break; }
  if (c->variant < 0) {
    wv_destroy(c);
    return fail(WV_EUNSUPPORTED, "no fused variant fits tile %d", desc->tile);
  }
  *out = c;
  return WV_OK;
}

wv_status wv_destroy(wv_ctx* c) {
  if (!c) return WV_OK;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  if (c->counter) hipFree(c->counter);
  if (c->plain_ws) hipFree(c->plain_ws);
  if (c->tab_dev) hipFree(c->tab_dev);
  if (c->tab_host) hipHostFree(c->tab_host);
  for (int i = 0; i < kTableSlots; ++i)
    if (c->tab_done[i]) hipEventDestroy(c->tab_done[i]);
  delete c;
  return WV_OK;
}

wv_status wv_set_path(wv_ctx* c, int32_t path) {
  g_err[0] = 0;
  if (!c) return fail(WV_EINVAL, "ctx is NULL");
  if (path != WV_PATH_FUSED && path != WV_PATH_PLAIN) return fail(WV_EINVAL, "bad path %d", path);
  if (path == WV_PATH_PLAIN && !c->plain_ws) {
    const size_t per_item = (size_t)c->d.tile * c->d.tile * (c->nplanes == 3 ? 3 : 2) / 2;
    const size_t bytes = 256 * per_item * 4;
    hipError_t e = hipMalloc(&c->plain_ws, bytes);
    if (e != hipSuccess) {
      c->plain_ws = nullptr;
      return fail(WV_ENOMEM, "plain workspace (%zu bytes): %s", bytes, hipGetErrorString(e));
    }
  }
  c->path = path;
  return WV_OK;
}

int32_t wv_variant_count(const wv_ctx* c) {
  return c ? fused_variant_count(c->d.wavelet, c->d.format) : 0;
}

wv_status wv_get_variant(const wv_ctx* c, int32_t* v) {
  if (!c || !v) return fail(WV_EINVAL, "NULL argument");
  *v = c->variant;
  return WV_OK;
}

wv_status wv_set_variant(wv_ctx* c, int32_t v) {
  if (!c) return fail(WV_EINVAL, "ctx is NULL");
  const Variant* var = fused_variant(c->d.wavelet, c->d.format, v);
  if (!var) return fail(WV_EINVAL, "variant %d out of range", v);
  if (!variant_fits(c->d, var)) return fail(WV_EUNSUPPORTED, "variant %s does not fit tile %d", var->name, c->d.tile);
  c->variant = v;
  return WV_OK;
}

const char* wv_variant_name(const wv_ctx* c, int32_t v) {
  if (!c) return "";
  const Variant* var = fused_variant(c->d.wavelet, c->d.format, v);
  return var ? var->name : "";
}

}  // extern "C"

// ------------------------------------------------------------ validation
struct JobPlan {
  std::vector<Item> items;   // visible tiles, ascending
};

wv_status wvp::check_job(const wv_ctx* c, const wv_frame* f, const uint8_t* mask, const wv_ref* ref,
                         const void* out, int job_index) {
  if (!c) return fail(WV_EINVAL, "job %d: ctx is NULL", job_index);
  if (!f || !mask || !ref) return fail(WV_EINVAL, "job %d: coeffs, tile_mask and ref are required", job_index);
  if (f->reserved != 0) return fail(WV_EINVAL, "job %d: wv_frame.reserved must be 0", job_index);
  if (!ref->tile_stamp) return fail(WV_EINVAL, "job %d: ref->tile_stamp is NULL", job_index);
  for (int p = 0; p < c->nplanes; ++p) {
    if (!f->planes[p] || !ref->planes[p])
      return fail(WV_EINVAL, "job %d: plane %d pointer is NULL", job_index, p);
    if (!aligned16(f->planes[p]) || !aligned16(ref->planes[p]))
      return fail(WV_EINVAL, "job %d: plane %d pointer is not 16-byte aligned", job_index, p);
  }
  if (out && !aligned16(out)) return fail(WV_EINVAL, "job %d: out is not 16-byte aligned", job_index);
  if (c->d.wavelet == WV_W53 && (f->qstep < 1 || f->qstep > 65535))
    return fail(WV_EINVAL, "job %d: qstep %d outside 1..65535", job_index, f->qstep);
  return WV_OK;
}

static wv_status validate_job(const wv_ctx* c, const wv_frame* f, const uint8_t* lc,
                              const uint8_t* mask, const wv_ref* ref, const void* out,
                              int job_index, JobPlan& plan) {
  wv_status st = check_job(c, f, mask, ref, out, job_index);
  if (st != WV_OK) return st;
  plan.items.clear();
  int slot = 0;
  for (int t = 0; t < c->n_tiles; ++t) {
    if (!mask[t]) continue;
    const int l = lc ? lc[t] : c->d.levels;
    if (l > c->d.levels)
      return fail(WV_EINVAL, "job %d: level_count[%d] = %d exceeds levels %d", job_index, t, l, c->d.levels);
    if (!f->is_intra && ref->tile_stamp[t] != f->frame_index - 1)
      return fail(WV_ESTALE, "job %d: tile %d has stamp %d, residual frame %d needs %d", job_index, t,
                  ref->tile_stamp[t], f->frame_index, f->frame_index - 1);
    Item it;
    it.tile = (uint16_t)t;
    it.slot = (uint16_t)slot++;
    it.job = 0;
    it.lc = (uint8_t)l;
    it.pad = 0;
    plan.items.push_back(it);
  }
  return WV_OK;
}

Job wvp::make_job(const wv_ctx* c, const wv_frame* f, const wv_ref* ref, void* out) {
  Job j = {};
  for (int p = 0; p < 3; ++p) {
    j.coef[p] = p < c->nplanes ? f->planes[p] : nullptr;
    j.ref[p] = p < c->nplanes ? ref->planes[p] : nullptr;
  }
  j.out = out;
  j.qstep = c->d.wavelet == WV_W53 ? f->qstep : 1;
  j.flags = (f->is_intra ? kJobIntra : 0u) | (out ? kJobHasOut : 0u);
  return j;
}

void wvp::fill_geometry(const wv_ctx* c, const Variant* var, WorkArgs& a) {
  a.tile = c->d.tile;
  a.levels = c->d.levels;
  a.bx = c->d.tile / var->bw;
  a.by = c->d.tile / var->bh;
  a.counter = c->counter;
  a.jobs_dev = nullptr;
  a.items_dev = nullptr;
}

// Launch a job list through kernel arguments, in chunks of kArgItems items.
static wv_status launch_arg_chunks(const wv_ctx* c, const Job* jobs, int n_jobs,
                                   const std::vector<Item>& items, hipStream_t s) {
  const Variant* var = fused_variant(c->d.wavelet, c->d.format, c->variant);
  WorkArgs a;
  memset(&a, 0, sizeof a);
  fill_geometry(c, var, a);
  for (int j = 0; j < n_jobs; ++j) a.jobs[j] = jobs[j];
  const int bpt = a.bx * a.by;
  for (size_t i0 = 0; i0 < items.size(); i0 += kArgItems) {
    const int n = (int)std::min<size_t>(kArgItems, items.size() - i0);
    std::copy(items.begin() + i0, items.begin() + i0 + n, a.items);
    a.n_items = n;
    a.total = n * bpt;
    hipError_t e = launch_fused(c->d.wavelet, c->d.format, c->variant, a, c->n_cu, s);
    if (e != hipSuccess) return hip_fail(e, "fused launch");
  }
  return WV_OK;
}

static wv_status launch_plain_items(wv_ctx* c, const Job& job, const std::vector<Item>& items,
                                    hipStream_t s) {
  PlainArgs a;
  memset(&a, 0, sizeof a);
  a.tile = c->d.tile;
  a.levels = c->d.levels;
  a.nplanes = c->nplanes;
  a.qstep = job.qstep;
  a.flags = job.flags;
  for (int p = 0; p < 3; ++p) {
    a.coef[p] = job.coef[p];
    a.ref[p] = job.ref[p];
  }
  a.out = job.out;
  a.ws = c->plain_ws;
  for (size_t i0 = 0; i0 < items.size(); i0 += 256) {
    const int n = (int)std::min<size_t>(256, items.size() - i0);
    std::copy(items.begin() + i0, items.begin() + i0 + n, a.items);
    a.n_items = n;
    hipError_t e = launch_plain(c->d.wavelet, c->d.format, a, s);
    if (e != hipSuccess) return hip_fail(e, "plain launch");
  }
  return WV_OK;
}

extern "C" wv_status wv_decode_viewport(wv_ctx* c, const wv_frame* f, const uint8_t* lc,
                                        const uint8_t* mask, wv_ref* ref, void* out,
                                        hipStream_t s) {
  g_err[0] = 0;
  JobPlan plan;
  wv_status st = validate_job(c, f, lc, mask, ref, out, 0, plan);
  if (st != WV_OK) return st;
  if (plan.items.empty()) return WV_OK;
  const Job job = make_job(c, f, ref, out);
  if (c->path == WV_PATH_PLAIN)
    st = launch_plain_items(c, job, plan.items, s);
  else
    st = launch_arg_chunks(c, &job, 1, plan.items, s);
  if (st != WV_OK) return st;
  for (const Item& it : plan.items) ref->tile_stamp[it.tile] = f->frame_index;
  return WV_OK;
}

extern "C" wv_status wv_decode_gop(wv_ctx* c, int32_t n_frames, const wv_frame* frames,
                                   const uint8_t* lc, const uint8_t* mask, wv_ref* ref,
                                   void* const* outs, hipStream_t s) {
  g_err[0] = 0;
  if (!c) return fail(WV_EINVAL, "ctx is NULL");
  if (n_frames < 1 || !frames) return fail(WV_EINVAL, "wv_decode_gop: need n_frames >= 1 frames");
  JobPlan plan;
  std::vector<Job> jobs(n_frames);
  for (int f = 0; f < n_frames; ++f) {
    if (frames[f].frame_index != frames[0].frame_index + f)
      return fail(WV_EINVAL, "wv_decode_gop: frame %d has index %d, expected %d", f, frames[f].frame_index,
                  frames[0].frame_index + f);
    void* out = outs ? outs[f] : nullptr;
    // the first frame is checked against the stamps; later ones follow it
    wv_status st = f == 0 ? validate_job(c, &frames[0], lc, mask, ref, out, 0, plan) : WV_OK;
    if (st != WV_OK) return st;
    if (f > 0) {
      JobPlan p2;
      wv_ref chained = *ref;
      std::vector<int32_t> stamps(c->n_tiles, frames[f].frame_index - 1);
      chained.tile_stamp = stamps.data();
      st = validate_job(c, &frames[f], lc, mask, &chained, out, f, p2);
      if (st != WV_OK) return st;
    }
    jobs[f] = make_job(c, &frames[f], ref, out);
  }
  if (plan.items.empty()) return WV_OK;
  const Variant* var = fused_variant(c->d.wavelet, c->d.format, c->variant);
  wv_status st = WV_OK;
  if (c->path == WV_PATH_FUSED && var->kind == 2) {
    // one launch per group of up to kArgJobs frames: each unit takes its tile
    // strip through the group's frames in order
    WorkArgs a;
    memset(&a, 0, sizeof a);
    fill_geometry(c, var, a);
    const int bpt = a.bx * a.by;
    for (int f0 = 0; f0 < n_frames && st == WV_OK; f0 += kArgJobs) {
      const int nf = std::min(kArgJobs, n_frames - f0);
      for (int j = 0; j < nf; ++j) a.jobs[j] = jobs[f0 + j];
      a.n_frames = nf;
      for (size_t i0 = 0; i0 < plan.items.size(); i0 += kArgItems) {
        const int n = (int)std::min<size_t>(kArgItems, plan.items.size() - i0);
        std::copy(plan.items.begin() + i0, plan.items.begin() + i0 + n, a.items);
        a.n_items = n;
        a.total = n * bpt;
        const hipError_t e = launch_fused(c->d.wavelet, c->d.format, c->variant, a, c->n_cu, s);
        if (e != hipSuccess) {
          st = hip_fail(e, "fused GOP launch");
          break;
        }
      }
    }
  } else {
    // other forms: one decode per frame
    for (int f = 0; f < n_frames && st == WV_OK; ++f)
      st = c->path == WV_PATH_PLAIN ? launch_plain_items(c, jobs[f], plan.items, s)
                                    : launch_arg_chunks(c, &jobs[f], 1, plan.items, s);
  }
  if (st != WV_OK) return st;
  for (const Item& it : plan.items) ref->tile_stamp[it.tile] = frames[n_frames - 1].frame_index;
  return WV_OK;
}

// Inter-frame sets (Section 3.2): frame t of a set is band 0 plus one signed
// detail band per Haar level; the strip kernels compiled for sets sum the
// three bands as they load them.
extern "C" wv_status wv_decode_set(wv_ctx* c, const wv_set* set, int32_t t0, int32_t n_frames,
                                   const uint8_t* lc, const uint8_t* mask, void* const* outs,
                                   hipStream_t s) {
  g_err[0] = 0;
  if (!c || !set || !mask || !outs)
    return fail(WV_EINVAL, "wv_decode_set: ctx, set, tile_mask and outs are required");
  if (set->n != 2 && set->n != 4)
    return fail(WV_EUNSUPPORTED, "wv_decode_set: sets of %d frames (2 or 4 supported)", set->n);
  if (n_frames < 1 || t0 < 0 || t0 + n_frames > set->n)
    return fail(WV_EINVAL, "wv_decode_set: frames %d .. %d outside a set of %d", t0, t0 + n_frames - 1,
                set->n);
  for (int p = 0; p < c->nplanes; ++p) {
    if (!set->planes[p]) return fail(WV_EINVAL, "wv_decode_set: plane %d pointer is NULL", p);
    if (!aligned16(set->planes[p]))
      return fail(WV_EINVAL, "wv_decode_set: plane %d pointer is not 16-byte aligned", p);
  }
  for (int f = 0; f < n_frames; ++f)
    if (!outs[f] || !aligned16(outs[f]))
      return fail(WV_EINVAL, "wv_decode_set: outs[%d] is NULL or not 16-byte aligned", f);
  const bool w53 = c->d.wavelet == WV_W53;
  if (w53)
    for (int b = 0; b < set->n; ++b)
      if (set->qstep[b] < 1 || set->qstep[b] > 65535)
        return fail(WV_EINVAL, "wv_decode_set: qstep[%d] = %d outside 1..65535", b, set->qstep[b]);
  // the context's variant if it is a row strip, else the first row strip that fits
  const Variant* var = fused_variant(c->d.wavelet, c->d.format, c->variant);
  if (!var || var->kind != 2) {
    var = nullptr;
    const int nv = fused_variant_count(c->d.wavelet, c->d.format);
    for (int v = 0; v < nv && !var; ++v) {
      const Variant* cand = fused_variant(c->d.wavelet, c->d.format, v);
      if (cand && cand->kind == 2 && variant_fits(c->d, cand)) var = cand;
    }
    if (!var)
      return fail(WV_EUNSUPPORTED, "wv_decode_set: no row-strip kernel for tile %d with %d levels",
                  c->d.tile, c->d.levels);
  }
  const size_t band = (size_t)c->n_tiles * c->d.tile * c->d.tile;
  if (band > 0xffffffffull) return fail(WV_EUNSUPPORTED, "wv_decode_set: bands of %zu samples", band);
  std::vector<Item> items;
  for (int t = 0; t < c->n_tiles; ++t) {
    if (!mask[t]) continue;
    const int l = lc ? lc[t] : c->d.levels;
    if (l > c->d.levels)
      return fail(WV_EINVAL, "wv_decode_set: level_count[%d] = %d exceeds levels %d", t, l, c->d.levels);
    Item it = {};
    it.tile = (uint16_t)t;
    it.slot = (uint16_t)items.size();
    it.lc = (uint8_t)l;
    items.push_back(it);
  }
  if (items.empty()) return WV_OK;
  WorkArgs a;
  memset(&a, 0, sizeof a);
  fill_geometry(c, var, a);
  for (int f = 0; f < n_frames; ++f) {
    const int t = t0 + f;
    Job& j = a.jobs[f];
    for (int p = 0; p < c->nplanes; ++p) j.coef[p] = set->planes[p];
    j.out = outs[f];
    j.qstep = w53 ? set->qstep[0] : 1;
    j.flags = kJobIntra | kJobHasOut;
    j.hstride = (uint32_t)band;
    // the coarsest detail (sign: the top bit of t) and, for sets of four,
    // the finest detail covering t (sign: bit 0)
    const int top = set->n == 4 ? (t >> 1) & 1 : t & 1;
    j.hq[0] = (top ? -1 : 1) * (w53 ? set->qstep[1] : 1);
    if (set->n == 4) {
      j.hband = 2 + (t >> 1);
      j.hq[1] = (t & 1 ? -1 : 1) * (w53 ? set->qstep[j.hband] : 1);
    } else {
      j.hband = 0;
      j.hq[1] = 0;
    }
  }
  a.n_frames = n_frames;
  const int bpt = a.bx * a.by;
  for (size_t i0 = 0; i0 < items.size(); i0 += kArgItems) {
    const int n = (int)std::min<size_t>(kArgItems, items.size() - i0);
    std::copy(items.begin() + i0, items.begin() + i0 + n, a.items);
    a.n_items = n;
    a.total = n * bpt;
    const hipError_t e = w53 ? launch_strip53_set(c->d.format, var->shape, var->levels, a, s)
                             : launch_strip97_set(c->d.format, var->shape, var->levels, a, s);
    if (e != hipSuccess) return hip_fail(e, "inter-frame set launch");
  }
  return WV_OK;
}

extern "C" wv_status wv_decode_batch(int32_t n_jobs, const wv_job* jobs, hipStream_t s) {
  g_err[0] = 0;
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(WV_EINVAL, "bad job list");
  if (n_jobs == 0) return WV_OK;
  if (n_jobs > kTableJobs) return fail(WV_EINVAL, "at most %d jobs per batch", kTableJobs);
  wv_ctx* c0 = jobs[0].ctx;
  if (!c0) return fail(WV_EINVAL, "job 0: ctx is NULL");
  std::vector<Job> table(n_jobs);
  std::vector<Item> items;
  JobPlan plan;
  for (int j = 0; j < n_jobs; ++j) {
    const wv_job& jb = jobs[j];
    wv_status st = validate_job(jb.ctx, jb.coeffs, jb.level_count, jb.tile_mask, jb.ref, jb.out, j, plan);
    if (st != WV_OK) return st;
    const wv_desc& d = jb.ctx->d;
    if (jb.ctx->device != c0->device || d.tile != c0->d.tile || d.levels != c0->d.levels ||
        d.wavelet != c0->d.wavelet || d.format != c0->d.format)
      return fail(WV_EUNSUPPORTED, "job %d: contexts in a batch must share device, tile, levels, wavelet, format", j);
    for (int k = 0; k < j; ++k)
      if (jobs[k].ref == jb.ref || (jobs[k].ref && jb.ref && jobs[k].ref->planes[0] == jb.ref->planes[0]))
        return fail(WV_EINVAL, "jobs %d and %d write the same reference", k, j);
    table[j] = make_job(jb.ctx, jb.coeffs, jb.ref, jb.out);
    for (Item it : plan.items) {
      it.job = (uint8_t)j;
      items.push_back(it);
    }
  }
  if ((int)items.size() > kTableItems) return fail(WV_EINVAL, "at most %d visible tiles per batch", kTableItems);
  if (!items.empty()) {
    const Variant* var = fused_variant(c0->d.wavelet, c0->d.format, c0->variant);
    if (n_jobs <= kArgJobs && (int)items.size() <= kArgItems) {
      wv_status st = launch_arg_chunks(c0, table.data(), n_jobs, items, s);
      if (st != WV_OK) return st;
    } else {
      // device table: stage in pinned memory, copy, launch once
      const int slot = c0->tab_next;
      c0->tab_next = (slot + 1) % kTableSlots;
      hipError_t e = hipEventSynchronize(c0->tab_done[slot]);
      if (e != hipSuccess) return hip_fail(e, "batch table wait");
      unsigned char* hst = c0->tab_host + slot * kTableBytes;
      unsigned char* dev = c0->tab_dev + slot * kTableBytes;
      memcpy(hst, table.data(), n_jobs * sizeof(Job));
      memcpy(hst + kTableJobs * sizeof(Job), items.data(), items.size() * sizeof(Item));
      e = hipMemcpyAsync(dev, hst, kTableJobs * sizeof(Job) + items.size() * sizeof(Item),
                         hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return hip_fail(e, "batch table copy");
      WorkArgs a;
      memset(&a, 0, sizeof a);
      fill_geometry(c0, var, a);
      a.jobs_dev = (const Job*)dev;
      a.items_dev = (const Item*)(dev + kTableJobs * sizeof(Job));
      a.n_items = (int)items.size();
      a.total = a.n_items * a.bx * a.by;
      e = launch_fused(c0->d.wavelet, c0->d.format, c0->variant, a, c0->n_cu, s);
      if (e != hipSuccess) return hip_fail(e, "fused batch launch");
      e = hipEventRecord(c0->tab_done[slot], s);
      if (e != hipSuccess) return hip_fail(e, "batch table event");
    }
  }
  for (int j = 0; j < n_jobs; ++j) {
    const wv_job& jb = jobs[j];
    for (int t = 0; t < jb.ctx->n_tiles; ++t)
      if (jb.tile_mask[t]) jb.ref->tile_stamp[t] = jb.coeffs->frame_index;
  }
  return WV_OK;
}

// ---------------------------------------------------------------- encoder
extern "C" wv_status wv_encode_intra(wv_ctx* c, const void* const* src, void* const* coeffs,
                                     int32_t qstep, hipStream_t s) {
  g_err[0] = 0;
  if (!c || !src || !coeffs) return fail(WV_EINVAL, "NULL argument");
  if (qstep < 1 || qstep > 65535) return fail(WV_EINVAL, "qstep %d outside 1..65535", qstep);
  for (int p = 0; p < c->nplanes; ++p)
    if (!src[p] || !coeffs[p]) return fail(WV_EINVAL, "plane %d pointer is NULL", p);
  const size_t vbytes = c->d.wavelet == WV_W53 ? 4 : 8;
  const size_t bytes = (size_t)c->n_tiles * c->d.tile * c->d.tile * vbytes;
  void* ws = nullptr;
  int* flag = nullptr;
  hipError_t e = hipMalloc(&ws, bytes);
  if (e != hipSuccess) return fail(WV_ENOMEM, "encoder workspace: %s", hipGetErrorString(e));
  e = hipMalloc((void**)&flag, sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(int), s);
  if (e == hipSuccess)
    e = launch_encode(c->d.wavelet, c->nplanes, c->n_tiles, c->d.tile, c->d.levels, qstep, src,
                      coeffs, ws, flag, s);
  int h_flag = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(ws);
  if (flag) hipFree(flag);
  if (e != hipSuccess) return hip_fail(e, "wv_encode_intra");
  if (h_flag) return fail(WV_EINVAL, "a quantisation index falls outside int16 (raise qstep)");
  return WV_OK;
}

// ------------------------------------------------------------------ tuner
extern "C" wv_status wv_autotune(wv_ctx* c, int32_t n_visible, int32_t reps, hipStream_t s,
                                 int32_t* best_variant) {
  g_err[0] = 0;
  if (!c) return fail(WV_EINVAL, "ctx is NULL");
  if (n_visible < 1 || n_visible > c->n_tiles || reps < 1)
    return fail(WV_EINVAL, "n_visible must be in 1..n_tiles and reps >= 1");
  const wv_desc& d = c->d;
  size_t cbytes[3], rbytes[3];
  void* cp[3] = {};
  void* rp[3] = {};
  void* out = nullptr;
  hipError_t e = hipSuccess;
  for (int p = 0; p < c->nplanes && e == hipSuccess; ++p) {
    const size_t P = plane_edge(d, p);
    cbytes[p] = (size_t)n_visible * P * P * coeff_bytes(d);
    rbytes[p] = (size_t)n_visible * P * P * sample_bytes(d);
    e = hipMalloc(&cp[p], cbytes[p]);
    if (e == hipSuccess) e = hipMalloc(&rp[p], rbytes[p]);
    if (e == hipSuccess) e = hipMemsetAsync(cp[p], 0, cbytes[p], s);
    if (e == hipSuccess) e = hipMemsetAsync(rp[p], 0, rbytes[p], s);
  }
  if (e == hipSuccess)
    e = hipMalloc(&out, (size_t)n_visible * c->nplanes * d.tile * d.tile * sample_bytes(d));
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  int best = -1;
  float best_ms = 1e30f;
  if (e == hipSuccess) {
    Job job = {};
    for (int p = 0; p < 3; ++p) {
      job.coef[p] = cp[p];
      job.ref[p] = rp[p];
    }
    job.out = out;
    job.qstep = 1;
    job.flags = kJobHasOut;
    std::vector<Item> items(n_visible);
    for (int i = 0; i < n_visible; ++i) items[i] = Item{(uint16_t)i, (uint16_t)i, 0, (uint8_t)d.levels, 0};
    const int saved = c->variant;
    for (int v = 0; v < wv_variant_count(c) && e == hipSuccess; ++v) {
      if (!variant_fits(d, fused_variant(d.wavelet, d.format, v))) continue;
      c->variant = v;
      wv_status st = WV_OK;
      for (int w = 0; w < 2 && st == WV_OK; ++w) st = launch_arg_chunks(c, &job, 1, items, s);
      if (st == WV_OK) e = hipEventRecord(t0, s);
      for (int r = 0; r < reps && st == WV_OK && e == hipSuccess; ++r)
        st = launch_arg_chunks(c, &job, 1, items, s);
      if (st != WV_OK) { e = hipErrorLaunchFailure; break; }
      if (e == hipSuccess) e = hipEventRecord(t1, s);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e == hipSuccess && ms < best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    c->variant = best >= 0 ? best : saved;
  }
  if (t0) hipEventDestroy(t0);
  if (t1) hipEventDestroy(t1);
  hipStreamSynchronize(s);
  for (int p = 0; p < 3; ++p) {
    if (cp[p]) hipFree(cp[p]);
    if (rp[p]) hipFree(rp[p]);
  }
  if (out) hipFree(out);
  if (e != hipSuccess) return hip_fail(e, "wv_autotune");
  if (best_variant) *best_variant = c->variant;
  return WV_OK;
}
