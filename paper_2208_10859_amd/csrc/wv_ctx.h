// Private to libwv: the context structure and helpers shared by the decode
// entry points (wv_api.cpp) and the serving loop (wv_server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "wv_internal.h"

namespace wvp {

wv_status fail(wv_status s, const char* fmt, ...);
wv_status hip_fail(hipError_t e, const char* what);
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
inline bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

constexpr int kTableSlots = 2;
constexpr int kTableJobs = 256;
constexpr int kTableItems = 16384;
constexpr size_t kTableBytes = kTableJobs * sizeof(wv::Job) + kTableItems * sizeof(wv::Item);

inline int plane_edge(const wv_desc& d, int p) { return p == 0 ? d.tile : d.tile / 2; }
inline size_t coeff_bytes(const wv_desc& d) { return d.wavelet == WV_W53 ? 2 : 4; }
inline size_t sample_bytes(const wv_desc& d) { return d.wavelet == WV_W53 ? 1 : 4; }
bool variant_fits(const wv_desc& d, const wv::Variant* v);

}  // namespace wvp

struct wv_ctx {
  wv_desc d;
  int device = 0;
  int n_cu = 256;
  int n_tiles = 0;
  int nplanes = 1;
  int path = WV_PATH_FUSED;
  int variant = 0;
  uint32_t* counter = nullptr;     // persistent-queue counters (device, 2 words)
  void* plain_ws = nullptr;        // plain-path workspace (device)
  // batch tables: pinned staging + device copy, double-buffered
  unsigned char* tab_host = nullptr;
  unsigned char* tab_dev = nullptr;
  hipEvent_t tab_done[wvp::kTableSlots] = {};
  int tab_next = 0;
};

namespace wvp {
wv_status check_desc(const wv_desc* d);
// argument checks of one decode job (pointers, alignment, qstep), no tiles
wv_status check_job(const wv_ctx* c, const wv_frame* f, const uint8_t* mask, const wv_ref* ref,
                    const void* out, int job_index);
wv::Job make_job(const wv_ctx* c, const wv_frame* f, const wv_ref* ref, void* out);
void fill_geometry(const wv_ctx* c, const wv::Variant* var, wv::WorkArgs& a);
}  // namespace wvp
