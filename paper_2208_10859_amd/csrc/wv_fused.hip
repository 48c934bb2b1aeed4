// Fused viewport decode for gfx950.
//
// One work unit = one luma output block (BW x BH) of one visible tile of one
// job, plus the co-located (BW/2 x BH/2) chroma blocks.  Tiles are
// transformed independently and the inverse lifting has a short support, so
// a block depends only on a small window of every level (its dependency
// cone).  Per block:
//
//  1. coarse levels (L .. 2) of each plane run in LDS on the cone windows,
//     ending in the level-2 output window W_2 (the approximation input of
//     the finest level);
//  2. the finest level runs in registers: each thread owns one output column
//     pair and TR consecutive rows; it lifts the rows its columns need
//     (approximation from W_2, details straight from the coefficient store),
//     then its two columns;
//  3. still in registers: residual onto the reference, clip, reference write,
//     and (luma threads, chroma read back from LDS) YUV420 -> RGB.
//
// No intermediate level touches HBM.  The only traffic is the coefficient
// windows, the reference block and the output block.
#include "wv_fused_common.h"

namespace wv {

// A coarse level task on plane state `ps` (level l, region edge n) whose
// computed window starts at (car, cac) with nr rows: the run of TRL rows
// starting q*TRL (the last run shifted back to end at the window's end).
template <class LF, int TRL, bool GEN, int PITCH, class CT>
__device__ __forceinline__ void coarse_task(PlaneState<CT, typename LF::V>& ps, int l, int L,
                                            int lc, int qstep, int q, int j, int car, int nr,
                                            int cac, int war, int wac, int war2, int wac2) {
  using V = typename LF::V;
  const int n = ps.P >> (l - 1);
  const int rr = car + min(q * TRL, nr - TRL), cc = cac + 2 * j;
  V o[TRL][2];
  level_task<LF, TRL, GEN, PITCH>(ps.in, war2, wac2, ps.coef, ps.lgP, n, l <= L - lc, qstep, rr,
                                  cc, o);
  V* dst = ps.out + (rr - war) * PITCH + (cc - wac);
#pragma unroll
  for (int i = 0; i < TRL; ++i) {
    dst[i * PITCH] = o[i][0];
    dst[i * PITCH + 1] = o[i][1];
  }
}

template <class LF, int FMT, int BW, int BH, int TR, bool GEN>
__device__ __forceinline__ void fused_unit(FusedSmem<LF, FMT, BW, BH>& sm, const WorkArgs& a, int unit) {
  using V = typename LF::V;
  using CT = typename CoefT<LF>::T;
  using RT = typename CoefT<LF>::R;
  using SM = FusedSmem<LF, FMT, BW, BH>;
  constexpr int NT = (BW / 2) * (BH / TR);
  constexpr int NP = FMT == WV_YUV420 ? 3 : 1;
  const int bpt = a.bx * a.by;
  const int it = unit / bpt, blk = unit - it * bpt;
  const Item item = a.items_dev ? a.items_dev[it] : a.items[it];
  const Job& job = a.jobs_dev ? a.jobs_dev[item.job] : a.jobs[item.job];
  const int T = a.tile, L = a.levels, lc = item.lc, qs = job.qstep;
  const int lgT = 31 - __clz(T);
  const int by = blk / a.bx, bx = blk - by * a.bx;
  const int r0 = by * BH, c0 = bx * BW;
  const bool intra = (job.flags & kJobIntra) != 0;
  const int tid = threadIdx.x;

  PlaneState<CT, V> ps[NP];
  {
    const WV_G CT* cy = uniform((const WV_G CT*)job.coef[0] + (size_t)item.tile * T * T);
    ps[0] = PlaneState<CT, V>{cy, T, lgT, r0, c0, BH, BW, sm.BY[0], sm.BY[1], SM::PY};
    if constexpr (NP == 3) {
      const int Pc = T >> 1;
      for (int p = 1; p < 3; ++p) {
        const WV_G CT* cp = uniform((const WV_G CT*)job.coef[p] + (size_t)item.tile * Pc * Pc);
        ps[p] = PlaneState<CT, V>{cp, Pc, lgT - 1, r0 >> 1, c0 >> 1, BH / 2, BW / 2, sm.BC[p - 1][0],
                                  sm.BC[p - 1][1], SM::PC};
      }
    }
  }

  // ---- approximation band windows W_{L+1} of every plane
  {
    int nr[NP], nc[NP], war[NP], wac[NP], sh[NP], slots = 0, start[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      int ca, cb, wb;
      level_window<LF>(L + 1, ps[p].P, L, ps[p].r0, ps[p].bh, ca, cb, war[p], wb);
      nr[p] = wb - war[p];
      level_window<LF>(L + 1, ps[p].P, L, ps[p].c0, ps[p].bw, ca, cb, wac[p], wb);
      nc[p] = wb - wac[p];
      sh[p] = ceil_log2(nc[p]);
      start[p] = slots;
      slots += nr[p] << sh[p];
    }
    for (int i = tid; i < slots; i += NT) {
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        if (i >= start[k] && (k + 1 == NP || i < start[k + 1])) {
          const int loc = i - start[k], r = loc >> sh[k], c = loc & ((1 << sh[k]) - 1);
          if (c < nc[k]) {
            const int nL = ps[k].P >> (L - 1);
            ps[k].in[r * ps[k].pitch + c] =
                deq(ldg(ps[k].coef, ((unsigned)sband<GEN>(war[k] + r, nL) << ps[k].lgP) +
                                        (unsigned)sband<GEN>(wac[k] + c, nL)),
                    qs);
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- coarse levels L .. 2, all planes per phase
  for (int l = L; l >= 2; --l) {
    int car[NP], nr[NP], cac[NP], ncw[NP], war[NP], wac[NP], wbr[NP], wbc[NP], war2[NP], wac2[NP];
    int sh[NP], start[NP], slots = 0;
    bool fill = false;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      int cb, t0, t1;
      level_window<LF>(l, ps[p].P, L, ps[p].r0, ps[p].bh, car[p], cb, war[p], wbr[p]);
      nr[p] = cb - car[p];
      fill |= war[p] != car[p] || wbr[p] != cb;
      level_window<LF>(l, ps[p].P, L, ps[p].c0, ps[p].bw, cac[p], cb, wac[p], wbc[p]);
      ncw[p] = cb - cac[p];
      fill |= wac[p] != cac[p] || wbc[p] != cb;
      level_window<LF>(l + 1, ps[p].P, L, ps[p].r0, ps[p].bh, t0, t1, war2[p], t1);
      level_window<LF>(l + 1, ps[p].P, L, ps[p].c0, ps[p].bw, t0, t1, wac2[p], t1);
      const int nrun = nr[p] >= 4 ? (nr[p] + 3) >> 2 : 1;
      sh[p] = ceil_log2(ncw[p] >> 1);
      start[p] = slots;
      slots += nrun << sh[p];
    }
    for (int i = tid; i < slots; i += NT) {
      auto plane_task = [&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int PT = k == 0 ? SM::PY : SM::PC;
        bool mine = i >= start[k];
        if constexpr (k + 1 < NP) mine = mine && i < start[k + 1];
        if (!mine) return;
        const int loc = i - start[k], q = loc >> sh[k], j = loc & ((1 << sh[k]) - 1);
        if (2 * j >= ncw[k]) return;
        if (nr[k] >= 4)
          coarse_task<LF, 4, GEN, PT>(ps[k], l, L, lc, qs, q, j, car[k], nr[k], cac[k], war[k],
                                      wac[k], war2[k], wac2[k]);
        else
          coarse_task<LF, 2, GEN, PT>(ps[k], l, L, lc, qs, q, j, car[k], nr[k], cac[k], war[k],
                                      wac[k], war2[k], wac2[k]);
      };
      plane_task(std::integral_constant<int, 0>{});
      if constexpr (NP == 3) {
        plane_task(std::integral_constant<int, 1>{});
        plane_task(std::integral_constant<int, 2>{});
      }
    }
    __syncthreads();
    if (fill) {
      // W_l outside the region: low-band mirror of the level l-1 signal
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        int ca, cb, cc0, cc1, t0, t1;
        level_window<LF>(l, ps[p].P, L, ps[p].r0, ps[p].bh, ca, cb, t0, t1);
        level_window<LF>(l, ps[p].P, L, ps[p].c0, ps[p].bw, cc0, cc1, t0, t1);
        const int nup = ps[p].P >> (l - 2);
        const int nwr = wbr[p] - war[p], nwc = wbc[p] - wac[p], s2 = ceil_log2(nwc);
        V* o = ps[p].out;
        const int pt = ps[p].pitch;
        for (int i = tid; i < (nwr << s2); i += NT) {
          const int r = i >> s2, c = i & ((1 << s2) - 1);
          const int gr = war[p] + r, gc = wac[p] + c;
          if (c < nwc && (gr < ca || gr >= cb || gc < cc0 || gc >= cc1))
            o[r * pt + c] = o[(sband<GEN>(gr, nup) - war[p]) * pt + (sband<GEN>(gc, nup) - wac[p])];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      V* t = ps[p].in;
      ps[p].in = ps[p].out;
      ps[p].out = t;
    }
  }

  const bool drop1 = 1 <= L - lc;
  // ---- finest chroma level (threads split between Cb and Cr), residual, clip
  if constexpr (NP == 3) {
    constexpr int TRC = TR / 2, CW = BW / 4;
    // Cb/Cr split: wave-uniform only when each half is a whole number of waves
    constexpr bool WAVE_UNIFORM = (NT / 2) % 64 == 0;
    const int pc = WAVE_UNIFORM ? __builtin_amdgcn_readfirstlane(tid / (NT / 2)) : tid / (NT / 2);
    const int t2 = tid - pc * (NT / 2);
    const int p2 = t2 % CW, q2 = t2 / CW;
    const int Pc = T >> 1;
    const int rr = (r0 >> 1) + q2 * TRC, cc = (c0 >> 1) + 2 * p2;
    int t0, t1, w2r, w2c;
    level_window<LF>(2, Pc, L, r0 >> 1, BH / 2, t0, t1, w2r, t1);
    level_window<LF>(2, Pc, L, c0 >> 1, BW / 2, t0, t1, w2c, t1);
    // per-thread plane choice (the two halves of the group take Cb and Cr)
    const V* w2 = pc ? ps[2].in : ps[1].in;
    const WV_G CT* ccoef = pc ? ps[2].coef : ps[1].coef;
    if constexpr (WAVE_UNIFORM) ccoef = uniform(ccoef);
    V o[TRC][2];
    level_task<LF, TRC, GEN, SM::PC>(w2, w2r, w2c, ccoef, lgT - 1, Pc, drop1, qs, rr, cc, o);
    WV_G RT* ref = (WV_G RT*)job.ref[1 + pc] + (size_t)item.tile * Pc * Pc;
    if constexpr (WAVE_UNIFORM) ref = uniform(ref);
    V* chr = sm.CHR + pc * (BH / 2) * (BW / 2);
#pragma unroll
    for (int i = 0; i < TRC; ++i) {
      WV_G RT* rp = at(ref, (unsigned)((rr + i) * Pc + cc));
      V a0 = o[i][0], a1 = o[i][1];
      if (!intra) {
        V b0, b1;
        load2(rp, b0, b1);
        a0 += b0;
        a1 += b1;
      }
      a0 = clip255(a0);
      a1 = clip255(a1);
      store2(rp, a0, a1);
      chr[(q2 * TRC + i) * (BW / 2) + 2 * p2] = a0;
      chr[(q2 * TRC + i) * (BW / 2) + 2 * p2 + 1] = a1;
    }
    __syncthreads();
  }

  // ---- finest luma level, residual, clip, colour
  {
    const int p = tid % (BW / 2), q = tid / (BW / 2);
    const int rr = r0 + q * TR, cc = c0 + 2 * p;
    int t0, t1, w2r, w2c;
    level_window<LF>(2, T, L, r0, BH, t0, t1, w2r, t1);
    level_window<LF>(2, T, L, c0, BW, t0, t1, w2c, t1);
    WV_G RT* ref = uniform((WV_G RT*)job.ref[0] + (size_t)item.tile * T * T);
    V o[TR][2];
    level_task<LF, TR, GEN, SM::PY>(ps[0].in, w2r, w2c, ps[0].coef, lgT, T, drop1, qs, rr, cc, o);
    const bool has_out = (job.flags & kJobHasOut) != 0;
    const size_t plane = (size_t)T * T;
    WV_G RT* out = uniform((WV_G RT*)job.out + (size_t)item.slot * NP * plane);
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const unsigned g = (unsigned)((rr + i) * T + cc);
      V y0 = o[i][0], y1 = o[i][1];
      if (!intra) {
        V b0, b1;
        load2(at(ref, g), b0, b1);
        y0 += b0;
        y1 += b1;
      }
      y0 = clip255(y0);
      y1 = clip255(y1);
      store2(at(ref, g), y0, y1);
      if (has_out) {
        if constexpr (NP == 3) {
          const int ci = ((q * TR + i) >> 1) * (BW / 2) + p;
          const V cb = sm.CHR[ci], cr = sm.CHR[(BH / 2) * (BW / 2) + ci];
          V R0, G0, B0, R1, G1, B1;
          to_rgb(y0, cb, cr, R0, G0, B0);
          to_rgb(y1, cb, cr, R1, G1, B1);
          store2(at(out, g), R0, R1);
          store2(at(out, g + (unsigned)plane), G0, G1);
          store2(at(out, g + 2u * (unsigned)plane), B0, B1);
        } else {
          store2(at(out, g), y0, y1);
        }
      }
    }
  }
  __syncthreads();
}

template <class LF, int FMT, int BW, int BH, int TR, bool PERSIST, bool GEN>
__global__ __launch_bounds__((BW / 2) * (BH / TR)) void k_fused(const WorkArgs a) {
  __shared__ FusedSmem<LF, FMT, BW, BH> sm;
  const int total = a.total_dev ? *a.total_dev : a.total;
  if (!PERSIST) {
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    if (u < total) fused_unit<LF, FMT, BW, BH, TR, GEN>(sm, a, u);
    return;
  }
  __shared__ int s_unit;
  for (;;) {
    if (threadIdx.x == 0) s_unit = (int)atomicAdd(&a.counter[0], 1u);
    __syncthreads();
    const int u = s_unit;
    __syncthreads();
    if (u >= total) break;
    fused_unit<LF, FMT, BW, BH, TR, GEN>(sm, a, u);
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

// ------------------------------------------------------------- variants
// General variants (runtime level count): block width, block height, rows
// per thread, persistent, groups per CU, general mirroring.  Variants without
// general mirroring need every mirrored region to have at least 16 samples:
// (plane edge >> (L-1)) >= 16.
#define WV_VARIANTS(X)                                 \
  X(64, 128, 16, false, 0, false, "b64x128_r16_grid")  \
  X(64, 64, 8, false, 0, false, "b64x64_r8_grid")      \
  X(128, 32, 8, false, 0, false, "b128x32_r8_grid")    \
  X(64, 64, 8, true, 5, false, "b64x64_r8_persist")    \
  X(64, 64, 8, false, 0, true, "b64x64_r8_general")    \
  X(32, 32, 8, false, 0, true, "b32x32_r8_general")    \
  X(16, 16, 4, false, 0, true, "b16x16_r4_general")         \
  X(32, 32, 8, true, 8, true, "b32x32_r8_general_persist")  \
  X(16, 16, 4, true, 8, true, "b16x16_r4_general_persist")

// Fast variants (compile-time level count, one staging phase per block):
// name, block width, block height, rows per thread, persistent, groups per
// CU, level count, shape index in the fast launcher.
#define WV_FAST_VARIANTS(X)                                   \
  X("fast_b64x64_r8_L5_grid", 64, 64, 8, false, 0, 5, 0)      \
  X("fast_b64x128_r16_L5_grid", 64, 128, 16, false, 0, 5, 1)  \
  X("fast_b128x32_r8_L5_grid", 128, 32, 8, false, 0, 5, 2)    \
  X("fast_b64x64_r8_L5_persist", 64, 64, 8, true, 4, 5, 0)    \
  X("fast_b64x64_r8_L4_grid", 64, 64, 8, false, 0, 4, 0)      \
  X("fast_b64x128_r16_L4_grid", 64, 128, 16, false, 0, 4, 1)  \
  X("fast_b128x32_r8_L4_grid", 128, 32, 8, false, 0, 4, 2)    \
  X("fast_b64x64_r8_L4_persist", 64, 64, 8, true, 4, 4, 0)    \
  X("fast_b64x64_r8_L3_grid", 64, 64, 8, false, 0, 3, 0)      \
  X("fast_b64x128_r16_L3_grid", 64, 128, 16, false, 0, 3, 1)  \
  X("fast_b128x32_r8_L3_grid", 128, 32, 8, false, 0, 3, 2)    \
  X("fast_b64x64_r8_L3_persist", 64, 64, 8, true, 4, 3, 0)

// Row-strip variants (512-sample tiles, compile-time level count): name,
// strip rows, waves, persistent, groups per CU, level count, shape index in
// the strip launcher.
#define WV_STRIP_VARIANTS(X) \
  X("strip_r32_w4_L5_grid", 32, 4, false, 0, 5, 0) \
  X("strip_r16_w4_L5_grid", 16, 4, false, 0, 5, 1) \
  X("strip_r32_w8_L5_grid", 32, 8, false, 0, 5, 2) \
  X("strip_r32_w4_L5_persist", 32, 4, true, 2, 5, 0) \
  X("strip_r16_w4_L5_persist", 16, 4, true, 3, 5, 1) \
  X("strip_r16_w4_L5_chain_persist", 16, 4, true, 5, 5, 4) \
  X("strip_r32_w4_L5_chain_grid", 32, 4, false, 0, 5, 3) \
  X("strip_r16_w4_L5_chain_grid", 16, 4, false, 0, 5, 4) \
  X("strip_r32_w4_L4_grid", 32, 4, false, 0, 4, 0) \
  X("strip_r16_w4_L4_grid", 16, 4, false, 0, 4, 1) \
  X("strip_r32_w8_L4_grid", 32, 8, false, 0, 4, 2) \
  X("strip_r32_w4_L4_persist", 32, 4, true, 2, 4, 0) \
  X("strip_r16_w4_L4_persist", 16, 4, true, 3, 4, 1) \
  X("strip_r16_w4_L4_chain_persist", 16, 4, true, 5, 4, 4) \
  X("strip_r32_w4_L4_chain_grid", 32, 4, false, 0, 4, 3) \
  X("strip_r16_w4_L4_chain_grid", 16, 4, false, 0, 4, 4) \
  X("strip_r32_w4_L3_grid", 32, 4, false, 0, 3, 0) \
  X("strip_r16_w4_L3_grid", 16, 4, false, 0, 3, 1) \
  X("strip_r32_w8_L3_grid", 32, 8, false, 0, 3, 2) \
  X("strip_r32_w4_L3_persist", 32, 4, true, 2, 3, 0) \
  X("strip_r16_w4_L3_persist", 16, 4, true, 3, 3, 1) \
  X("strip_r16_w4_L3_chain_persist", 16, 4, true, 5, 3, 4) \
  X("strip_r32_w4_L3_chain_grid", 32, 4, false, 0, 3, 3) \
  X("strip_r16_w4_L3_chain_grid", 16, 4, false, 0, 3, 4)

// Strip variants come first, then the fast block variants: the default
// variant of a context is the first one that fits its geometry.
static const Variant kVariants[] = {
#define WV_S(name, r, nw, pers, gpc, lv, shape) \
  {name, 512, r, 64 * nw, pers, gpc, false, lv, shape, 2, -1, -1},
    WV_STRIP_VARIANTS(WV_S)
#undef WV_S
#define WV_F(name, bw, bh, tr, pers, gpc, lv, shape) \
  {name, bw, bh, (bw / 2) * (bh / tr), pers, gpc, false, lv, shape, 1, -1, -1},
    WV_FAST_VARIANTS(WV_F)
#undef WV_F
#define WV_V(bw, bh, tr, pers, gpc, gen, name) \
  {name, bw, bh, (bw / 2) * (bh / tr), pers, gpc, gen, 0, -1, 0, -1, -1},
    WV_VARIANTS(WV_V)
#undef WV_V
};
#define WV_ONE(...) +1
static constexpr int kNumSpecial = 0 WV_STRIP_VARIANTS(WV_ONE) WV_FAST_VARIANTS(WV_ONE);
#undef WV_ONE
static constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int fused_variant_count(int, int) { return kNumVariants; }
const Variant* fused_variant(int, int, int v) {
  return (v >= 0 && v < kNumVariants) ? &kVariants[v] : nullptr;
}

template <class LF, int FMT>
static hipError_t launch_fused_t(int v, const WorkArgs& a, int n_cu, hipStream_t s) {
  int idx = kNumSpecial;
#define WV_L(bw, bh, tr, pers, gpc, gen, name)                                             \
  if (v == idx) {                                                                        \
    const int grid = pers ? min(a.total, n_cu * gpc) : a.total;                          \
    if (grid <= 0) return hipSuccess;                                                    \
    hipLaunchKernelGGL((k_fused<LF, FMT, bw, bh, tr, pers, gen>), dim3(grid),            \
                       dim3((bw / 2) * (bh / tr)), 0, s, a);                             \
    return hipGetLastError();                                                            \
  }                                                                                      \
  ++idx;
  WV_VARIANTS(WV_L)
#undef WV_L
  const Variant* var = fused_variant(0, FMT, v);
  if (!var || var->levels == 0) return hipErrorInvalidValue;
  if (var->kind == 2)
    return std::is_same<LF, Inv53>::value
               ? launch_strip53(FMT, var->shape, var->levels, var->persistent, a, n_cu, s)
               : launch_strip97(FMT, var->shape, var->levels, var->persistent, a, n_cu, s);
  if (std::is_same<LF, Inv53>::value)
    return launch_fast53(FMT, var->shape, var->levels, var->persistent, a, n_cu, s);
  return launch_fast97(FMT, var->shape, var->levels, var->persistent, a, n_cu, s);
}

hipError_t launch_fused(int wavelet, int format, int v, const WorkArgs& a, int n_cu,
                        hipStream_t s) {
  if (wavelet == WV_W53)
    return format == WV_YUV420 ? launch_fused_t<Inv53, WV_YUV420>(v, a, n_cu, s)
                               : launch_fused_t<Inv53, WV_GRAY8>(v, a, n_cu, s);
  return format == WV_YUV420 ? launch_fused_t<Inv97, WV_YUV420>(v, a, n_cu, s)
                             : launch_fused_t<Inv97, WV_GRAY8>(v, a, n_cu, s);
}

}  // namespace wv
