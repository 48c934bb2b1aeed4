// The sparse storage format (Sections 3.3, 3.4, 3.6): host encoder, and the
// entry point of the GPU rebuild (Section 3.5).  The encoder is offline work,
// as in the paper: plain host code, one plane of one frame per call.
#include <algorithm>
#include <cmath>
#include <cstring>
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
