// HIP kernels for gfx950: the fused viewport decode, the plain per-step
// decode, and the intra encoder used to build coefficient stores.
//
// Fused form.  One work unit = one luma output block (BW x BH) of one visible
// tile of one job, plus the co-located chroma blocks.  Tiles are transformed
// independently, and the inverse lifting has a short support, so an output
// block depends only on a small window of every level (its dependency
// cone): the group loads those coefficient windows (with symmetric extension
// at tile edges), runs every level's rows-then-columns inverse inside LDS,
// and finishes the block in the same pass (residual onto the reference,
// clip, reference write, YUV420 -> RGB).  No intermediate level ever goes to
// HBM: the only traffic is the coefficient windows, the reference block and
// the output block.
#include "wv_internal.h"
#include "wv_lift.h"

namespace wv {

// ----------------------------------------------------------------- helpers
constexpr int kMaxTile = 512;
__device__ __forceinline__ int floor_even(int x) { return x & ~1; }
__device__ __forceinline__ int ceil_even(int x) { return (x + 1) & ~1; }

template <class LF>
struct CoefT;
template <>
struct CoefT<Inv53> { using T = int16_t; using R = uint8_t; };
template <>
struct CoefT<Inv97> { using T = float; using R = float; };

__device__ __forceinline__ int deq(int16_t q, int step) { return (int)q * step; }
__device__ __forceinline__ float deq(float q, int) { return q; }

__device__ __forceinline__ int clip255(int v) { return min(max(v, 0), 255); }
__device__ __forceinline__ float clip255(float v) { return fminf(fmaxf(v, 0.0f), 255.0f); }

// YUV -> RGB, JFIF full range.  Integer: Q16 constants round(65536 k).
__device__ __forceinline__ void to_rgb(int y, int cb, int cr, int& r, int& g, int& b) {
  cb -= 128;
  cr -= 128;
  r = clip255(((y << 16) + 91881 * cr + 32768) >> 16);
  g = clip255(((y << 16) - 22554 * cb - 46802 * cr + 32768) >> 16);
  b = clip255(((y << 16) + 116130 * cb + 32768) >> 16);
}
__device__ __forceinline__ void to_rgb(float y, float cb, float cr, float& r, float& g,
                                       float& b) {
  cb -= 128.0f;
  cr -= 128.0f;
  r = clip255(y + 1.402f * cr);
  g = clip255(y - 0.344136f * cb - 0.714136f * cr);
  b = clip255(y + 1.772f * cb);
}

// Level windows of a block, one dimension.  Level 1's computed window C_1
// is the block itself.  Level k needs the low-band samples
// [C_k.a/2 - S_LO, C_k.b/2 + S_HI) of level k+1's output; that range rounded
// out to even bounds is the layout window W_{k+1} (kept in LDS), and the part
// of it inside the level k+1 region [0, P >> k) is what level k+1 computes,
// C_{k+1}.  The rest of W_{k+1} lies outside the region and is filled by
// mirroring: the low band of a whole-sample-symmetric signal is itself
// symmetric about its first sample on the left and about the point between
// its last two samples on the right, which differs from the extension a
// coarser level's output would get on its own -- so those samples are
// copied, never computed.  The approximation band (level L+1) is stored:
// its whole window W_{L+1} is loaded with that mirroring.
template <class LF>
__device__ __forceinline__ void level_window(int k, int P, int L, int a1, int n1, int& ca, int& cb,
                                             int& wa, int& wb) {
  ca = a1;
  cb = a1 + n1;
  wa = ca;
  wb = cb;
  for (int j = 1; j < k; ++j) {
    wa = floor_even((ca >> 1) - LF::S_LO);
    wb = ceil_even((cb >> 1) + LF::S_HI);
    if (j + 1 <= L) {
      ca = max(wa, 0);
      cb = min(wb, P >> j);
    } else {
      ca = wa;
      cb = wb;
    }
  }
}

// Compile-time bound of every level's window length for a level-1 block of B.
template <class LF>
constexpr int win_max(int B) {
  int len = B, mx = B;
  for (int k = 0; k < 14; ++k) {
    int nxt = len / 2 + LF::S_LO + LF::S_HI + 2;
    nxt += nxt & 1;
    if (nxt > mx) mx = nxt;
    len = nxt;
  }
  return mx;
}

__device__ __forceinline__ int xcd_remap(int b, int g) {
  // Work groups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous range of work units so neighbouring blocks of one tile (which
  // share coefficient halos) meet in the same L2.
  const int X = 8;
  const int q = g / X, r = g % X, x = b % X, i = b / X;
  return x * q + min(x, r) + i;
}

// ------------------------------------------------------------- fused kernel
template <class LF, int FMT, int BW, int BH>
struct FusedSmem {
  using V = typename LF::V;
  static constexpr int MR = win_max<LF>(BH), MC = win_max<LF>(BW);
  static constexpr int PA = MC + 1;
  static constexpr int NSR = MR / 2 + LF::S_LO + LF::S_HI, NDR = MR / 2 + LF::D_LO + LF::D_HI;
  static constexpr int NSC = MC / 2 + LF::S_LO + LF::S_HI, NDC = MC / 2 + LF::D_LO + LF::D_HI;
  static constexpr int PS = NSC + 1, PD = NDC + 1;
  static constexpr int NCHR = (FMT == WV_YUV420) ? 2 * (BH / 2) * (BW / 2) : 1;
  V A[MR * PA];      // LL input of the current level, then its output window
  V HL[NSR * PD];    // detail windows of the current level
  V LH[NDR * PS];
  V HH[NDR * PD];
  V TOP[NSR * PA];   // rows after the horizontal pass (low rows, high rows)
  V BOT[NDR * PA];
  V CHR[NCHR];       // reconstructed chroma of the block, for the colour step
};

// Inverse transform of one plane's block into sm.A ([bh][bw], pitch PA).
template <class LF, int NT, class SM>
__device__ void reconstruct_block(SM& sm, const typename CoefT<LF>::T* __restrict__ coef, int P,
                                  int L, int lc, int qstep, int r0, int c0, int bh, int bw) {
  using V = typename LF::V;
  constexpr int PA = SM::PA, PS = SM::PS, PD = SM::PD;
  const int tid = threadIdx.x;
  {
    // approximation band window W_{L+1} (low band of level L in both directions)
    const int n_L = P >> (L - 1);
    int ca, cb, wa_r, wb_r, wa_c, wb_c;
    level_window<LF>(L + 1, P, L, r0, bh, ca, cb, wa_r, wb_r);
    level_window<LF>(L + 1, P, L, c0, bw, ca, cb, wa_c, wb_c);
    const int nr2 = wb_r - wa_r, nc2 = wb_c - wa_c;
    for (int i = tid; i < nr2 * nc2; i += NT) {
      const int r = i / nc2, c = i - r * nc2;
      const int gr = s_idx(wa_r + r, n_L), gc = s_idx(wa_c + c, n_L);
      sm.A[r * PA + c] = deq(coef[gr * P + gc], qstep);
    }
  }
  for (int l = L; l >= 1; --l) {
    const int n_l = P >> (l - 1), h = n_l >> 1;
    int car, cbr, war, wbr, cac, cbc, wac, wbc, t0, t1, war2, wac2;
    level_window<LF>(l, P, L, r0, bh, car, cbr, war, wbr);
    level_window<LF>(l, P, L, c0, bw, cac, cbc, wac, wbc);
    level_window<LF>(l + 1, P, L, r0, bh, t0, t1, war2, t1);
    level_window<LF>(l + 1, P, L, c0, bw, t0, t1, wac2, t1);
    const int nr = cbr - car, nc = cbc - cac;
    const int sr0 = (car >> 1) - LF::S_LO, nsr = (nr >> 1) + LF::S_LO + LF::S_HI;
    const int dr0 = (car >> 1) - LF::D_LO, ndr = (nr >> 1) + LF::D_LO + LF::D_HI;
    const int sc0 = (cac >> 1) - LF::S_LO, nsc = (nc >> 1) + LF::S_LO + LF::S_HI;
    const int dc0 = (cac >> 1) - LF::D_LO, ndc = (nc >> 1) + LF::D_LO + LF::D_HI;
    if (l <= L - lc) {
      // foveation: this level's details are zero and are not read
      for (int i = tid; i < nsr * ndc; i += NT) {
        const int r = i / ndc, c = i - r * ndc;
        sm.HL[r * PD + c] = V(0);
      }
      for (int i = tid; i < ndr * nsc; i += NT) {
        const int r = i / nsc, c = i - r * nsc;
        sm.LH[r * PS + c] = V(0);
      }
      for (int i = tid; i < ndr * ndc; i += NT) {
        const int r = i / ndc, c = i - r * ndc;
        sm.HH[r * PD + c] = V(0);
      }
    } else {
      for (int i = tid; i < nsr * ndc; i += NT) {
        const int r = i / ndc, c = i - r * ndc;
        const int gr = s_idx(sr0 + r, n_l), gc = h + d_idx(dc0 + c, n_l);
        sm.HL[r * PD + c] = deq(coef[gr * P + gc], qstep);
      }
      for (int i = tid; i < ndr * nsc; i += NT) {
        const int r = i / nsc, c = i - r * nsc;
        const int gr = h + d_idx(dr0 + r, n_l), gc = s_idx(sc0 + c, n_l);
        sm.LH[r * PS + c] = deq(coef[gr * P + gc], qstep);
      }
      for (int i = tid; i < ndr * ndc; i += NT) {
        const int r = i / ndc, c = i - r * ndc;
        const int gr = h + d_idx(dr0 + r, n_l), gc = h + d_idx(dc0 + c, n_l);
        sm.HH[r * PD + c] = deq(coef[gr * P + gc], qstep);
      }
    }
    __syncthreads();
    // horizontal pass: low rows (LL | HL) -> TOP, high rows (LH | HH) -> BOT
    const int npc = nc >> 1;
    const int aoff_r = sr0 - war2, aoff_c = sc0 - wac2;
    for (int i = tid; i < (nsr + ndr) * npc; i += NT) {
      const int r = i / npc, j = i - r * npc;
      V s[LF::NS], d[LF::ND];
      V* dst;
      if (r < nsr) {
        const V* sp = &sm.A[(aoff_r + r) * PA + aoff_c + j];
        const V* dp = &sm.HL[r * PD + j];
#pragma unroll
        for (int t = 0; t < LF::NS; ++t) s[t] = sp[t];
#pragma unroll
        for (int t = 0; t < LF::ND; ++t) d[t] = dp[t];
        dst = &sm.TOP[r * PA + 2 * j];
      } else {
        const int rr = r - nsr;
        const V* sp = &sm.LH[rr * PS + j];
        const V* dp = &sm.HH[rr * PD + j];
#pragma unroll
        for (int t = 0; t < LF::NS; ++t) s[t] = sp[t];
#pragma unroll
        for (int t = 0; t < LF::ND; ++t) d[t] = dp[t];
        dst = &sm.BOT[rr * PA + 2 * j];
      }
      V xe, xo;
      LF::pair(s, d, xe, xo);
      dst[0] = xe;
      dst[1] = xo;
    }
    __syncthreads();
    // vertical pass: TOP (low) + BOT (high) -> computed window C_l of A
    // (layout W_l)
    const int npr = nr >> 1;
    const int or_ = car - war, oc = cac - wac;
    for (int i = tid; i < nc * npr; i += NT) {
      const int j = i / nc, c = i - j * nc;
      V s[LF::NS], d[LF::ND];
#pragma unroll
      for (int t = 0; t < LF::NS; ++t) s[t] = sm.TOP[(j + t) * PA + c];
#pragma unroll
      for (int t = 0; t < LF::ND; ++t) d[t] = sm.BOT[(j + t) * PA + c];
      V xe, xo;
      LF::pair(s, d, xe, xo);
      sm.A[(or_ + 2 * j) * PA + oc + c] = xe;
      sm.A[(or_ + 2 * j + 1) * PA + oc + c] = xo;
    }
    __syncthreads();
    if (l > 1 && (war != car || wbr != cbr || wac != cac || wbc != cbc)) {
      // fill the part of W_l outside the region by low-band mirroring
      const int n_up = P >> (l - 2);
      const int nwr = wbr - war, nwc = wbc - wac;
      for (int i = tid; i < nwr * nwc; i += NT) {
        const int r = i / nwc, c = i - r * nwc;
        const int gr = war + r, gc = wac + c;
        if (gr >= car && gr < cbr && gc >= cac && gc < cbc) continue;
        const int mr = s_idx(gr, n_up), mc = s_idx(gc, n_up);
        sm.A[r * PA + c] = sm.A[(mr - war) * PA + (mc - wac)];
      }
      __syncthreads();
    }
  }
}

template <class LF, int FMT, int BW, int BH, int NT>
__device__ void fused_unit(FusedSmem<LF, FMT, BW, BH>& sm, const WorkArgs& a, int unit) {
  using V = typename LF::V;
  using CT = typename CoefT<LF>::T;
  using RT = typename CoefT<LF>::R;
  using SM = FusedSmem<LF, FMT, BW, BH>;
  constexpr int PA = SM::PA;
  const int bpt = a.bx * a.by;
  const int it = unit / bpt, blk = unit - it * bpt;
  const Item item = a.items_dev ? a.items_dev[it] : a.items[it];
  const Job& job = a.jobs_dev ? a.jobs_dev[item.job] : a.jobs[item.job];
  const int T = a.tile, L = a.levels;
  const int by = blk / a.bx, bx = blk - by * a.bx;
  const int r0 = by * BH, c0 = bx * BW;
  const bool intra = (job.flags & kJobIntra) != 0;
  const int tid = threadIdx.x;

  if (FMT == WV_YUV420) {
    const int Pc = T >> 1;
    for (int p = 1; p <= 2; ++p) {
      const CT* coef = (const CT*)job.coef[p] + (size_t)item.tile * Pc * Pc;
      RT* ref = (RT*)job.ref[p] + (size_t)item.tile * Pc * Pc;
      reconstruct_block<LF, NT>(sm, coef, Pc, L, item.lc, job.qstep, r0 >> 1, c0 >> 1, BH / 2,
                                BW / 2);
      V* chr = &sm.CHR[(p - 1) * (BH / 2) * (BW / 2)];
      for (int i = tid; i < (BH / 2) * (BW / 2); i += NT) {
        const int r = i / (BW / 2), c = i - r * (BW / 2);
        const size_t g = (size_t)((r0 >> 1) + r) * Pc + (c0 >> 1) + c;
        const V pv = sm.A[r * PA + c];
        const V rec = clip255(intra ? pv : (V)ref[g] + pv);
        ref[g] = (RT)rec;
        chr[i] = rec;
      }
      __syncthreads();
    }
  }
  {
    const CT* coef = (const CT*)job.coef[0] + (size_t)item.tile * T * T;
    RT* ref = (RT*)job.ref[0] + (size_t)item.tile * T * T;
    reconstruct_block<LF, NT>(sm, coef, T, L, item.lc, job.qstep, r0, c0, BH, BW);
    const bool has_out = (job.flags & kJobHasOut) != 0;
    RT* out = (RT*)job.out;
    const size_t plane = (size_t)T * T;
    for (int i = tid; i < BH * BW; i += NT) {
      const int r = i / BW, c = i - r * BW;
      const size_t g = (size_t)(r0 + r) * T + c0 + c;
      const V pv = sm.A[r * PA + c];
      const V y = clip255(intra ? pv : (V)ref[g] + pv);
      ref[g] = (RT)y;
      if (has_out) {
        if (FMT == WV_YUV420) {
          const int ci = (r >> 1) * (BW / 2) + (c >> 1);
          V R, G, B;
          to_rgb(y, sm.CHR[ci], sm.CHR[(BH / 2) * (BW / 2) + ci], R, G, B);
          RT* o = out + (size_t)item.slot * 3 * plane + g;
          o[0] = (RT)R;
          o[plane] = (RT)G;
          o[2 * plane] = (RT)B;
        } else {
          out[(size_t)item.slot * plane + g] = (RT)y;
        }
      }
    }
    __syncthreads();
  }
}

template <class LF, int FMT, int BW, int BH, int NT, bool PERSIST>
__global__ __launch_bounds__(NT) void k_fused(const WorkArgs a) {
  __shared__ FusedSmem<LF, FMT, BW, BH> sm;
  if (!PERSIST) {
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    if (u < a.total) fused_unit<LF, FMT, BW, BH, NT>(sm, a, u);
    return;
  }
  __shared__ int s_unit;
  for (;;) {
    if (threadIdx.x == 0) s_unit = (int)atomicAdd(&a.counter[0], 1u);
    __syncthreads();
    const int u = s_unit;
    __syncthreads();
    if (u >= a.total) break;
    fused_unit<LF, FMT, BW, BH, NT>(sm, a, u);
  }
  // The last group to leave resets the queue for the next launch on this
  // stream: every group has made its final fetch before it counts itself out.
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned done = atomicAdd(&a.counter[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&a.counter[0], 0u);
      atomicExch(&a.counter[1], 0u);
    }
  }
}

// ----------------------------------------------------------- fused variants
#define WV_VARIANTS(X)                            \
  X(64, 64, 256, false, 0, "b64x64_t256_grid")    \
  X(64, 32, 256, false, 0, "b64x32_t256_grid")    \
  X(32, 32, 256, false, 0, "b32x32_t256_grid")    \
  X(128, 32, 256, false, 0, "b128x32_t256_grid")  \
  X(16, 16, 64, false, 0, "b16x16_t64_grid")      \
  X(64, 64, 256, true, 2, "b64x64_t256_persist")  \
  X(64, 32, 256, true, 3, "b64x32_t256_persist")  \
  X(32, 32, 256, true, 4, "b32x32_t256_persist")

static const Variant kVariants[] = {
#define WV_V(bw, bh, nt, pers, gpc, name) {name, bw, bh, nt, pers, gpc},
    WV_VARIANTS(WV_V)
#undef WV_V
};
static constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int fused_variant_count(int, int) { return kNumVariants; }
const Variant* fused_variant(int, int, int v) {
  return (v >= 0 && v < kNumVariants) ? &kVariants[v] : nullptr;
}

template <class LF, int FMT>
static hipError_t launch_fused_t(int v, const WorkArgs& a, int n_cu, hipStream_t s) {
  int idx = 0;
#define WV_L(bw, bh, nt, pers, gpc, name)                                       \
  if (v == idx) {                                                             \
    int grid = pers ? min(a.total, n_cu * gpc) : a.total;                     \
    if (grid <= 0) return hipSuccess;                                         \
    hipLaunchKernelGGL((k_fused<LF, FMT, bw, bh, nt, pers>), dim3(grid), dim3(nt), 0, s, a); \
    return hipGetLastError();                                                 \
  }                                                                           \
  ++idx;
  WV_VARIANTS(WV_L)
#undef WV_L
  return hipErrorInvalidValue;
}

hipError_t launch_fused(int wavelet, int format, int v, const WorkArgs& a, int n_cu,
                        hipStream_t s) {
  if (wavelet == WV_W53)
    return format == WV_YUV420 ? launch_fused_t<Inv53, WV_YUV420>(v, a, n_cu, s)
                               : launch_fused_t<Inv53, WV_GRAY8>(v, a, n_cu, s);
  return format == WV_YUV420 ? launch_fused_t<Inv97, WV_YUV420>(v, a, n_cu, s)
                             : launch_fused_t<Inv97, WV_GRAY8>(v, a, n_cu, s);
}

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
