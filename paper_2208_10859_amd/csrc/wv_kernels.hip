// HIP kernels for gfx950: the plain per-step decode (one launch per step
// and level through an HBM workspace) and the intra encoder used to build
// coefficient stores.
#include "wv_dev.h"
#include "wv_internal.h"

namespace wv {

// ============================================================== plain path
// Workspace: per item, the item's planes back to back as V (int32 / float).
__device__ __forceinline__ size_t plane_off(int p, int T) {
  // luma T*T, then chroma (T/2)^2 each
  return p == 0 ? 0 : (size_t)T * T + (size_t)(p - 1) * (T / 2) * (T / 2);
}

template <class LF>
__global__ __launch_bounds__(256) void k_plain_gather(const PlainArgs a) {
  using V = typename LF::V;
  using CT = typename CoefT<LF>::T;
  const int T = a.tile;
  const size_t per_item = a.nplanes == 3 ? (size_t)T * T * 3 / 2 : (size_t)T * T;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= per_item) return;
  const Item it = a.items[blockIdx.y];
  int p, P;
  size_t off;
  if (e < (size_t)T * T) { p = 0; P = T; off = e; }
  else {
    const size_t q = e - (size_t)T * T;
    P = T / 2;
    p = 1 + (int)(q / ((size_t)P * P));
    off = q - (size_t)(p - 1) * P * P;
  }
  const int r = (int)(off / P), c = (int)(off - (size_t)r * P);
  const CT q = ((const CT*)a.coef[p])[(size_t)it.tile * P * P + off];
  V v = deq(q, a.qstep);
  const int m = max(r, c);
  if (m >= (P >> a.levels)) {
    // detail sample: level = log2(P) - floor(log2(m)) (1 = finest)
    const int lev = (31 - __clz(P)) - (31 - __clz(m));
    if (lev <= a.levels - it.lc) v = V(0);
  }
  V* ws = (V*)a.ws + (size_t)blockIdx.y * per_item;
  ws[e] = v;
}

// One level, one direction, in place over the workspace.  Rows: each group
// owns RPW rows; columns: each group owns CPW adjacent columns.
template <class LF, bool ROWS>
__global__ __launch_bounds__(256) void k_plain_level(const PlainArgs a, int l) {
  using V = typename LF::V;
  constexpr int RPW = 4, CPW = 16;
  __shared__ V line[ROWS ? RPW * kMaxTile : kMaxTile * CPW];
  const int T = a.tile;
  const int item = blockIdx.y / a.nplanes, p = blockIdx.y - item * a.nplanes;
  const int P = p == 0 ? T : T / 2;
  const int n = P >> (l - 1), h = n >> 1;
  const size_t per_item = a.nplanes == 3 ? (size_t)T * T * 3 / 2 : (size_t)T * T;
  V* ws = (V*)a.ws + (size_t)item * per_item + plane_off(p, T);
  const int tid = threadIdx.x;
  const int nl = ROWS ? RPW : CPW;
  const int l0 = blockIdx.x * nl;
  if (l0 >= n) return;
  const int cnt = min(nl, n - l0);
  // load lines
  for (int i = tid; i < cnt * n; i += 256) {
    if (ROWS) {
      const int r = i / n, c = i - r * n;
      line[r * n + c] = ws[(size_t)(l0 + r) * P + c];
    } else {
      const int r = i / cnt, c = i - r * cnt;
      line[r * CPW + c] = ws[(size_t)r * P + l0 + c];
    }
  }
  __syncthreads();
  for (int i = tid; i < cnt * h; i += 256) {
    int ln, j;
    if (ROWS) { ln = i / h; j = i - ln * h; }
    else { j = i / cnt; ln = i - j * cnt; }
    V s[LF::NS], d[LF::ND];
#pragma unroll
    for (int t = 0; t < LF::NS; ++t) {
      const int k = s_idx(j - LF::S_LO + t, n);
      s[t] = ROWS ? line[ln * n + k] : line[k * CPW + ln];
    }
#pragma unroll
    for (int t = 0; t < LF::ND; ++t) {
      const int k = h + d_idx(j - LF::D_LO + t, n);
      d[t] = ROWS ? line[ln * n + k] : line[k * CPW + ln];
    }
    V xe, xo;
    LF::pair(s, d, xe, xo);
    if (ROWS) {
      ws[(size_t)(l0 + ln) * P + 2 * j] = xe;
      ws[(size_t)(l0 + ln) * P + 2 * j + 1] = xo;
    } else {
      ws[(size_t)(2 * j) * P + l0 + ln] = xe;
      ws[(size_t)(2 * j + 1) * P + l0 + ln] = xo;
    }
  }
}

template <class LF>
__global__ __launch_bounds__(256) void k_plain_residual(const PlainArgs a) {
  using V = typename LF::V;
  using RT = typename CoefT<LF>::R;
  const int T = a.tile;
  const size_t per_item = a.nplanes == 3 ? (size_t)T * T * 3 / 2 : (size_t)T * T;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= per_item) return;
  const Item it = a.items[blockIdx.y];
  int p, P;
  size_t off;
  if (e < (size_t)T * T) { p = 0; P = T; off = e; }
  else {
    const size_t q = e - (size_t)T * T;
    P = T / 2;
    p = 1 + (int)(q / ((size_t)P * P));
    off = q - (size_t)(p - 1) * P * P;
  }
  const V* ws = (const V*)a.ws + (size_t)blockIdx.y * per_item;
  RT* ref = (RT*)a.ref[p] + (size_t)it.tile * P * P + off;
  const V pv = ws[e];
  const V rec = clip255((a.flags & kJobIntra) ? pv : (V)*ref + pv);
  *ref = (RT)rec;
}

template <class LF, int FMT>
__global__ __launch_bounds__(256) void k_plain_colour(const PlainArgs a) {
  using V = typename LF::V;
  using RT = typename CoefT<LF>::R;
  const int T = a.tile;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t plane = (size_t)T * T;
  if (e >= plane) return;
  const Item it = a.items[blockIdx.y];
  const int r = (int)(e / T), c = (int)(e - (size_t)r * T);
  const RT* y = (const RT*)a.ref[0] + (size_t)it.tile * plane;
  RT* out = (RT*)a.out;
  if (FMT == WV_YUV420) {
    const int Pc = T / 2;
    const size_t ce = (size_t)(r >> 1) * Pc + (c >> 1);
    const RT* cb = (const RT*)a.ref[1] + (size_t)it.tile * Pc * Pc;
    const RT* cr = (const RT*)a.ref[2] + (size_t)it.tile * Pc * Pc;
    V R, G, B;
    to_rgb((V)y[e], (V)cb[ce], (V)cr[ce], R, G, B);
    RT* o = out + (size_t)it.slot * 3 * plane + e;
    o[0] = (RT)R;
    o[plane] = (RT)G;
    o[2 * plane] = (RT)B;
  } else {
    out[(size_t)it.slot * plane + e] = y[e];
  }
}

template <class LF, int FMT>
static hipError_t launch_plain_t(const PlainArgs& a, hipStream_t s) {
  const int T = a.tile;
  const size_t per_item = a.nplanes == 3 ? (size_t)T * T * 3 / 2 : (size_t)T * T;
  const dim3 ge((unsigned)((per_item + 255) / 256), (unsigned)a.n_items);
  hipLaunchKernelGGL(k_plain_gather<LF>, ge, dim3(256), 0, s, a);
  for (int l = a.levels; l >= 1; --l) {
    const int n = T >> (l - 1);
    hipLaunchKernelGGL((k_plain_level<LF, true>), dim3((n + 3) / 4, a.n_items * a.nplanes),
                       dim3(256), 0, s, a, l);
    hipLaunchKernelGGL((k_plain_level<LF, false>), dim3((n + 15) / 16, a.n_items * a.nplanes),
                       dim3(256), 0, s, a, l);
  }
  hipLaunchKernelGGL(k_plain_residual<LF>, ge, dim3(256), 0, s, a);
  if (a.out) {
    const dim3 gc((unsigned)(((size_t)T * T + 255) / 256), (unsigned)a.n_items);
    hipLaunchKernelGGL((k_plain_colour<LF, FMT>), gc, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_plain(int wavelet, int format, const PlainArgs& a, hipStream_t s) {
  if (wavelet == WV_W53)
    return format == WV_YUV420 ? launch_plain_t<Inv53, WV_YUV420>(a, s)
                               : launch_plain_t<Inv53, WV_GRAY8>(a, s);
  return format == WV_YUV420 ? launch_plain_t<Inv97, WV_YUV420>(a, s)
                             : launch_plain_t<Inv97, WV_GRAY8>(a, s);
}

// ================================================================= encoder
template <class V>
__global__ __launch_bounds__(256) void k_enc_load(const uint8_t* __restrict__ src,
                                                  V* __restrict__ ws, size_t n) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) ws[e] = (V)src[e];
}

// One forward level, one direction, in place: each group owns lines of one
// tile (rows: 4 rows; columns: 16 adjacent columns).
template <class LF, bool ROWS>
__global__ __launch_bounds__(256) void k_enc_level(typename LF::V* __restrict__ ws, int P,
                                                   int l) {
  using V = typename LF::V;
  constexpr int RPW = 4, CPW = sizeof(V) == 8 ? 8 : 16;
  __shared__ V line[ROWS ? RPW * kMaxTile : kMaxTile * CPW];
  const int n = P >> (l - 1), h = n >> 1;
  V* t = ws + (size_t)blockIdx.y * P * P;
  const int nl = ROWS ? RPW : CPW;
  const int l0 = blockIdx.x * nl;
  if (l0 >= n) return;
  const int cnt = min(nl, n - l0);
  const int tid = threadIdx.x;
  for (int i = tid; i < cnt * n; i += 256) {
    if (ROWS) {
      const int r = i / n, c = i - r * n;
      line[r * n + c] = t[(size_t)(l0 + r) * P + c];
    } else {
      const int r = i / cnt, c = i - r * cnt;
      line[r * CPW + c] = t[(size_t)r * P + l0 + c];
    }
  }
  __syncthreads();
  for (int i = tid; i < cnt * h; i += 256) {
    int ln, k;
    if (ROWS) { ln = i / h; k = i - ln * h; }
    else { k = i / cnt; ln = i - k * cnt; }
    auto x = [&](int j) -> V {
      const int q = wss(j, n);
      return ROWS ? line[ln * n + q] : line[q * CPW + ln];
    };
    V s, d;
    LF::pair(x, k, s, d);
    if (ROWS) {
      t[(size_t)(l0 + ln) * P + k] = s;
      t[(size_t)(l0 + ln) * P + h + k] = d;
    } else {
      t[(size_t)k * P + l0 + ln] = s;
      t[(size_t)(h + k) * P + l0 + ln] = d;
    }
  }
}

__global__ __launch_bounds__(256) void k_enc_quant53(const int* __restrict__ ws,
                                                     int16_t* __restrict__ dst, size_t n,
                                                     int step, int* overflow) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int c = ws[e];
  const int a = (2 * abs(c) + step) / (2 * step);
  const int q = c < 0 ? -a : a;
  if (q < -32768 || q > 32767) atomicOr(overflow, 1);
  dst[e] = (int16_t)q;
}

__global__ __launch_bounds__(256) void k_enc_quant97(const double* __restrict__ ws,
                                                     float* __restrict__ dst, size_t n,
                                                     int step) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double c = ws[e];
  const double a = floor(fabs(c) / step + 0.5);
  dst[e] = (float)(step * (c < 0 ? -a : a));
}

template <class LF>
static hipError_t launch_encode_t(int nplanes, int n_tiles, int tile, int levels, int qstep,
                                  const void* const* src, void* const* dst, void* ws,
                                  int* overflow, hipStream_t s) {
  using V = typename LF::V;
  for (int p = 0; p < nplanes; ++p) {
    const int P = p == 0 ? tile : tile / 2;
    const size_t n = (size_t)n_tiles * P * P;
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_enc_load<V>, dim3(g), dim3(256), 0, s, (const uint8_t*)src[p], (V*)ws,
                       n);
    for (int l = 1; l <= levels; ++l) {
      const int m = P >> (l - 1);
      const int cpw = sizeof(V) == 8 ? 8 : 16;
      hipLaunchKernelGGL((k_enc_level<LF, false>), dim3((m + cpw - 1) / cpw, n_tiles), dim3(256), 0, s,
                         (V*)ws, P, l);
      hipLaunchKernelGGL((k_enc_level<LF, true>), dim3((m + 3) / 4, n_tiles), dim3(256), 0, s,
                         (V*)ws, P, l);
    }
    if (sizeof(V) == 4)
      hipLaunchKernelGGL(k_enc_quant53, dim3(g), dim3(256), 0, s, (const int*)ws,
                         (int16_t*)dst[p], n, qstep, overflow);
    else
      hipLaunchKernelGGL(k_enc_quant97, dim3(g), dim3(256), 0, s, (const double*)ws,
                         (float*)dst[p], n, qstep);
  }
  return hipGetLastError();
}

hipError_t launch_encode(int wavelet, int nplanes, int n_tiles, int tile, int levels, int qstep,
                         const void* const* src, void* const* dst, void* ws, int* overflow,
                         hipStream_t s) {
  if (wavelet == WV_W53)
    return launch_encode_t<Fwd53>(nplanes, n_tiles, tile, levels, qstep, src, dst, ws, overflow,
                                  s);
  return launch_encode_t<Fwd97>(nplanes, n_tiles, tile, levels, qstep, src, dst, ws, overflow, s);
}

}  // namespace wv
