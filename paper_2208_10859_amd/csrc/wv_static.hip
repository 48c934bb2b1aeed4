// wv_decode_viewport_noalloc: the viewport decode of wv_decode_viewport for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  It needs no
// context: the geometry comes as a wv_desc, and the only device memory its
// kernels use beyond the caller's buffers -- the work-queue counters of the
// persistent decode kernels -- is a file-scope device array of this library.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "wv_ctx.h"

namespace {

// The persistent kernels' queue counters: [0] next work unit, [1] finished
// workgroups.  Each GPU holds its own copy until the process ends.
constexpr int kScratchWords = 64;   // 256 bytes; two are used
__device__ __align__(256) uint32_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
uint32_t* g_scratch[kMaxDevices];   // per device: the array's device address
std::mutex g_scratch_mu;

// The host-side name `scratch` is not a device address: the address is taken
// once per device with that device current, and only it is passed on.
wv_status scratch_address(int device, uint32_t** out) {
  if (device < 0 || device >= kMaxDevices)
    return wvp::fail(WV_EUNSUPPORTED, "device %d beyond %d devices", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return wvp::hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[device] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch[device];
  return WV_OK;
}

// Clears the counters stream-ordered (a kernel, not a memset node, so that a
// captured graph replays it faithfully).
__global__ void k_clear_counters(uint32_t* c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0u;
}

}  // namespace

extern "C" wv_status wv_decode_viewport_noalloc(const wv_desc* desc, const wv_frame* f,
                                               const uint8_t* lc, const uint8_t* mask,
                                               wv_ref* ref, void* out, hipStream_t s) {
  using namespace wv;
  wv_status st = wvp::check_desc(desc);
  if (st != WV_OK) return st;
  // a context on the stack: geometry only, no buffers
  wv_ctx c;
  c.d = *desc;
  c.n_tiles = (desc->width / desc->tile) * (desc->height / desc->tile);
  c.nplanes = desc->format == WV_YUV420 ? 3 : 1;
  hipError_t e = hipGetDevice(&c.device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c.n_cu, hipDeviceAttributeMultiprocessorCount, c.device);
  if (e != hipSuccess) return wvp::hip_fail(e, "wv_decode_viewport_noalloc: device query");
  c.variant = -1;
  for (int v = 0; v < fused_variant_count(desc->wavelet, desc->format); ++v) {
    const Variant* var = fused_variant(desc->wavelet, desc->format, v);
    if (var->persistent && wvp::variant_fits(c.d, var)) {
      c.variant = v;
      break;
    }
  }
  if (c.variant < 0) return wvp::fail(WV_EUNSUPPORTED, "no persistent fused variant fits this geometry");
  st = wvp::check_job(&c, f, mask, ref, out, 0);
  if (st != WV_OK) return st;
  // every visible tile is checked before anything is enqueued
  int n_vis = 0;
  for (int t = 0; t < c.n_tiles; ++t) {
    if (!mask[t]) continue;
    const int l = lc ? lc[t] : desc->levels;
    if (l > desc->levels)
      return wvp::fail(WV_EINVAL, "level_count[%d] = %d exceeds levels %d", t, l, desc->levels);
    if (!f->is_intra && ref->tile_stamp[t] != f->frame_index - 1)
      return wvp::fail(WV_ESTALE, "tile %d has stamp %d, residual frame %d needs %d", t, ref->tile_stamp[t],
                       f->frame_index, f->frame_index - 1);
    ++n_vis;
  }
  if (n_vis == 0) return WV_OK;
  uint32_t* counters = nullptr;
  st = scratch_address(c.device, &counters);
  if (st != WV_OK) return st;
  const Variant* var = fused_variant(desc->wavelet, desc->format, c.variant);
  WorkArgs a;
  std::memset(&a, 0, sizeof a);
  wvp::fill_geometry(&c, var, a);
  a.counter = counters;
  a.jobs[0] = wvp::make_job(&c, f, ref, out);
  const int bpt = a.bx * a.by;
  // items in ascending tile order, in chunks of the kernel-argument table
  int slot = 0, t = 0;
  while (slot < n_vis) {
    int n = 0;
    for (; t < c.n_tiles && n < kArgItems; ++t) {
      if (!mask[t]) continue;
      Item& it = a.items[n++];
      it.tile = (uint16_t)t;
      it.slot = (uint16_t)slot++;
      it.job = 0;
      it.lc = (uint8_t)(lc ? lc[t] : desc->levels);
      it.pad = 0;
    }
    a.n_items = n;
    a.total = n * bpt;
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, s, counters);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_fused(desc->wavelet, desc->format, c.variant, a, c.n_cu, s);
    if (e != hipSuccess) return wvp::hip_fail(e, "wv_decode_viewport_noalloc launch");
  }
  for (int k = 0; k < c.n_tiles; ++k)
    if (mask[k]) ref->tile_stamp[k] = f->frame_index;
  return WV_OK;
}
