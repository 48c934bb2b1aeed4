// Fast fused decode: the level count L is a compile-time constant.
//
// Same decomposition as the general fused kernel (one luma block plus its
// chroma blocks per work unit, dependency-cone windows per level), organised
// so that each block waits on memory once:
//
//  1. window geometry of every level is computed once (unrolled scalar code);
//  2. every detail window of the coarse levels (L .. 2) and the approximation
//     window are loaded in one batch -- all loads issued before any is used --
//     and staged in LDS (raw coefficients; dequantised on use); the reference
//     samples of the thread's output are fetched at the same time;
//  3. coarse levels run from LDS only; a level's output window is written
//     together with its mirror images outside the region (the low-band
//     symmetric extension), so no separate fill pass or barrier is needed;
//  4. the finest level runs in registers as in the general form, then
//     residual, clip, reference write and colour.
#pragma once

#include "wv_fused_common.h"

namespace wv {

template <class LF>
constexpr int fast_mxlo() { return LF::S_LO > LF::D_LO ? LF::S_LO : LF::D_LO; }
template <class LF>
constexpr int fast_mxhi() { return LF::S_HI > LF::D_HI ? LF::S_HI : LF::D_HI; }
// staged rows/cols of level l's detail windows for a block edge B
template <class LF>
constexpr int fast_nu(int B, int l) { return w_at<LF>(B, l) / 2 + fast_mxlo<LF>() + fast_mxhi<LF>(); }

template <class LF, int FMT, int BW, int BH, int L>
struct FastSmem {
  using V = typename LF::V;
  using CT = typename CoefT<LF>::T;
  static constexpr int MXLO = fast_mxlo<LF>(), MXHI = fast_mxhi<LF>();
  static constexpr int nu(int B, int l) { return fast_nu<LF>(B, l); }
  static constexpr int lvl_size(int BR, int BC, int l) { return 3 * nu(BR, l) * nu(BC, l); }
  static constexpr int lvl_off(int BR, int BC, int l) {
    int s = 0;
    for (int k = 2; k < l; ++k) s += lvl_size(BR, BC, k);
    return s;
  }
  static constexpr int NDY = lvl_off(BH, BW, L + 1), NDC = lvl_off(BH / 2, BW / 2, L + 1);
  static constexpr int RY = w_max_from<LF>(BH, 2), CY = w_max_from<LF>(BW, 2), PY = (CY + 3) & ~3;
  static constexpr int RC = w_max_from<LF>(BH / 2, 2), CC = w_max_from<LF>(BW / 2, 2),
                       PC = (CC + 3) & ~3;
  static constexpr int NCP = FMT == WV_YUV420 ? 2 : 0;
  CT detY[NDY > 0 ? NDY : 1];
  CT detC[NCP > 0 ? NCP : 1][NDC > 0 && NCP > 0 ? NDC : 1];
  V BY[2][RY * PY];
  V BC[NCP > 0 ? NCP : 1][2][NCP > 0 ? RC * PC : 1];
  V CHR[NCP > 0 ? NCP * (BH / 2) * (BW / 2) : 1];
};

// Window geometry of one dimension of a plane block for levels 1 .. L+1:
// computed window C = [ca, cb) and layout window W = [wa, wb).
template <class LF, int L>
struct Win1D {
  int ca[L + 2], cb[L + 2], wa[L + 2], wb[L + 2];
};
template <class LF, int L>
__device__ __forceinline__ void make_win(Win1D<LF, L>& w, int a1, int n1, int P) {
  w.ca[1] = a1;
  w.cb[1] = a1 + n1;
  w.wa[1] = a1;
  w.wb[1] = a1 + n1;
#pragma unroll
  for (int j = 1; j <= L; ++j) {
    w.wa[j + 1] = floor_even((w.ca[j] >> 1) - LF::S_LO);
    w.wb[j + 1] = ceil_even((w.cb[j] >> 1) + LF::S_HI);
    if (j + 1 <= L) {
      w.ca[j + 1] = max(w.wa[j + 1], 0);
      w.cb[j + 1] = min(w.wb[j + 1], P >> j);
    } else {
      w.ca[j + 1] = w.wa[j + 1];
      w.cb[j + 1] = w.wb[j + 1];
    }
  }
}

// Values of one plane's staging loads, held in registers between the load
// and the store phase.
template <class LF, class CT, int BHp, int BWp, int L, int NT>
struct StageVals {
  static constexpr int RL = w_at<LF>(BHp, L + 1), CL = w_at<LF>(BWp, L + 1);
  static constexpr int KL = (RL * CL + NT - 1) / NT;
  static constexpr int KMAX = (3 * fast_nu<LF>(BHp, 2) * fast_nu<LF>(BWp, 2) + NT - 1) / NT;
  CT vl[KL];
  CT vd[L > 1 ? L - 1 : 1][KMAX];
};

// Uniform geometry of one plane type's block (luma, or both chroma planes).
template <class LF, int L>
struct FastGeo {
  int P, lgP;
  Win1D<LF, L> wr, wc;
};

// One coarse-level task reading staged details: output columns cc, cc+1 and
// TRL rows from rr of level l (region edge m).  `in` holds level l+1's
// layout window (origin wr2/wc2), `det` the staged [HL | LH | HH] windows of
// level l (origin ur0/uc0, NUR x NUC each).  Outputs are written to `out`
// (layout window origin war/wac, end wbr/wbc) together with their low-band
// mirror images -u and 2m-1-u that fall inside the layout window.
template <class LF, int TRL, int PITCH, int NUR, int NUC, class CT>
__device__ __forceinline__ void staged_task(const typename LF::V* __restrict__ in, int wr2, int wc2,
                                            const CT* __restrict__ det, int ur0, int uc0,
                                            int qs, int rr, int cc, typename LF::V* __restrict__ out,
                                            int war, int wac, int wbr, int wbc, int m) {
  using V = typename LF::V;
  constexpr int NPR = TRL / 2;
  constexpr int NSV = NPR + LF::S_LO + LF::S_HI, NDV = NPR + LF::D_LO + LF::D_HI;
  constexpr int NSH = 1 + LF::S_LO + LF::S_HI, NDH = 1 + LF::D_LO + LF::D_HI;
  const int sr0 = (rr >> 1) - LF::S_LO, dr0 = (rr >> 1) - LF::D_LO;
  const int sc0 = (cc >> 1) - LF::S_LO, dc0 = (cc >> 1) - LF::D_LO;
  const CT* hl = det + (sr0 - ur0) * NUC + (dc0 - uc0);
  const CT* lh = det + (NUR + dr0 - ur0) * NUC + (sc0 - uc0);
  const CT* hh = det + (2 * NUR + dr0 - ur0) * NUC + (dc0 - uc0);
  const V* ll = in + (sr0 - wr2) * PITCH + (sc0 - wc2);
  V top[NSV][2], bot[NDV][2];
#pragma unroll
  for (int i = 0; i < NSV; ++i) {
    V s[NSH], d[NDH], x[2];
#pragma unroll
    for (int j = 0; j < NSH; ++j) s[j] = ll[i * PITCH + j];
#pragma unroll
    for (int j = 0; j < NDH; ++j) d[j] = deq(hl[i * NUC + j], qs);
    LF::template run<1>(s, d, x);
    top[i][0] = x[0];
    top[i][1] = x[1];
  }
#pragma unroll
  for (int i = 0; i < NDV; ++i) {
    V s[NSH], d[NDH], x[2];
#pragma unroll
    for (int j = 0; j < NSH; ++j) s[j] = deq(lh[i * NUC + j], qs);
#pragma unroll
    for (int j = 0; j < NDH; ++j) d[j] = deq(hh[i * NUC + j], qs);
    LF::template run<1>(s, d, x);
    bot[i][0] = x[0];
    bot[i][1] = x[1];
  }
  // column mirror images (same for every row of the task)
  int cimg[2][3];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int u = cc + c;
    cimg[c][0] = u - wac;
    cimg[c][1] = (u >= 1 && -u >= wac) ? -u - wac : -1;
    cimg[c][2] = (2 * m - 1 - u < wbc) ? 2 * m - 1 - u - wac : -1;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    V s[NSV], d[NDV], x[TRL];
#pragma unroll
    for (int i = 0; i < NSV; ++i) s[i] = top[i][c];
#pragma unroll
    for (int i = 0; i < NDV; ++i) d[i] = bot[i][c];
    LF::template run<NPR>(s, d, x);
#pragma unroll
    for (int i = 0; i < TRL; ++i) {
      const int u = rr + i;
      const int ri[3] = {u - war, (u >= 1 && -u >= war) ? -u - war : -1,
                         (2 * m - 1 - u < wbr) ? 2 * m - 1 - u - war : -1};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          if (ri[a] >= 0 && cimg[c][b] >= 0) out[ri[a] * PITCH + cimg[c][b]] = x[i];
    }
  }
}

// Two adjacent reference samples, kept packed until use.
__device__ __forceinline__ uint32_t load_raw2(const WV_G uint8_t* p) {
  return *(const WV_G uint16_t*)p;
}
__device__ __forceinline__ float2 load_raw2(const WV_G float* p) { return make_float2(p[0], p[1]); }
__device__ __forceinline__ void unpack2(uint32_t v, int& a, int& b) {
  a = v & 0xff;
  b = (v >> 8) & 0xff;
}
__device__ __forceinline__ void unpack2(float2 v, float& a, float& b) {
  a = v.x;
  b = v.y;
}

template <class LF, int FMT, int BW, int BH, int TR, int L>
__device__ __forceinline__ void fast_unit(FastSmem<LF, FMT, BW, BH, L>& sm, const WorkArgs& a, int unit) {
  using V = typename LF::V;
  using CT = typename CoefT<LF>::T;
  using RT = typename CoefT<LF>::R;
  using SM = FastSmem<LF, FMT, BW, BH, L>;
  constexpr int NT = (BW / 2) * (BH / TR);
  constexpr int NP = FMT == WV_YUV420 ? 3 : 1;
  constexpr int MXLO = SM::MXLO, MXHI = SM::MXHI;
  const int bpt = a.bx * a.by;
  const int it = unit / bpt, blk = unit - it * bpt;
  const Item item = a.items_dev ? a.items_dev[it] : a.items[it];
  const Job& job = a.jobs_dev ? a.jobs_dev[item.job] : a.jobs[item.job];
  const int T = a.tile, lc = item.lc, qs = job.qstep;
  const int lgT = 31 - __clz(T);
  const int by = blk / a.bx, bx = blk - by * a.bx;
  const int r0 = by * BH, c0 = bx * BW;
  const bool intra = (job.flags & kJobIntra) != 0;
  const bool drop1 = 1 <= L - lc;
  const int tid = threadIdx.x;

  // plane geometry: [0] luma, [1] both chroma planes (identical windows)
  constexpr int NG = NP == 3 ? 2 : 1;
  FastGeo<LF, L> geo[NG];
  geo[0].P = T;
  geo[0].lgP = lgT;
  make_win(geo[0].wr, r0, BH, T);
  make_win(geo[0].wc, c0, BW, T);
  const WV_G CT* coefs[NP];
  coefs[0] = uniform((const WV_G CT*)job.coef[0] + (size_t)item.tile * T * T);
  if constexpr (NP == 3) {
    geo[1].P = T >> 1;
    geo[1].lgP = lgT - 1;
    make_win(geo[1].wr, r0 >> 1, BH / 2, T >> 1);
    make_win(geo[1].wc, c0 >> 1, BW / 2, T >> 1);
#pragma unroll
    for (int p = 1; p < 3; ++p)
      coefs[p] = uniform((const WV_G CT*)job.coef[p] + (size_t)item.tile * (T >> 1) * (T >> 1));
  }

  // thread roles of the finest level
  const int lp = tid % (BW / 2), lq = tid / (BW / 2);
  const int lrr = r0 + lq * TR, lcc = c0 + 2 * lp;
  constexpr int TRC = TR / 2, CW = BW / 4;
  constexpr bool WAVE_UNIFORM = (NT / 2) % 64 == 0;
  const int pc = NP == 3 ? (WAVE_UNIFORM ? __builtin_amdgcn_readfirstlane(tid / (NT / 2))
                                         : tid / (NT / 2))
                         : 0;
  const int t2 = tid - pc * (NT / 2);
  const int cp2 = t2 % CW, cq2 = t2 / CW;
  const int crr = (r0 >> 1) + cq2 * TRC, ccc = (c0 >> 1) + 2 * cp2;

  // reference samples of the thread's outputs, fetched up front
  WV_G RT* refY = uniform((WV_G RT*)job.ref[0] + (size_t)item.tile * T * T);
  // packed: two adjacent samples per word for 8-bit references
  using RP = typename std::conditional<std::is_same<RT, uint8_t>::value, uint32_t, float2>::type;
  RP ry[TR];
  RP rc[TRC];
  WV_G RT* refC = nullptr;
  if constexpr (NP == 3) {
    refC = (WV_G RT*)job.ref[1 + pc] + (size_t)item.tile * (T >> 1) * (T >> 1);
    if constexpr (WAVE_UNIFORM) refC = uniform(refC);
  }
#pragma unroll
  for (int i = 0; i < TR; ++i) ry[i] = RP{};
#pragma unroll
  for (int i = 0; i < TRC; ++i) rc[i] = RP{};
  if (!intra) {
#pragma unroll
    for (int i = 0; i < TR; ++i) ry[i] = load_raw2(at(refY, (unsigned)((lrr + i) * T + lcc)));
    if constexpr (NP == 3) {
#pragma unroll
      for (int i = 0; i < TRC; ++i)
        rc[i] = load_raw2(at(refC, (unsigned)((crr + i) * (T >> 1) + ccc)));
    }
  }

  // ---- stage: approximation windows and every coarse detail window of all
  // planes; every load is issued before the first store
  StageVals<LF, CT, BH, BW, L, NT> sv0;
  StageVals<LF, CT, BH / 2, BW / 2, L, NT> sv1, sv2;
  auto load_plane = [&](auto pcst, auto& sv) {
    constexpr int p = decltype(pcst)::value;
    constexpr int BHp = p == 0 ? BH : BH / 2, BWp = p == 0 ? BW : BW / 2;
    using SV = std::remove_reference_t<decltype(sv)>;
    const FastGeo<LF, L>& P_ = geo[p > 0 ? 1 : 0];
    const WV_G CT* pcoef = coefs[p];
    const int nL = P_.P >> (L - 1);
    const int lr0 = P_.wr.wa[L + 1], lc0 = P_.wc.wa[L + 1];
    const int lnr = P_.wr.wb[L + 1] - lr0, lnc = P_.wc.wb[L + 1] - lc0;
#pragma unroll
    for (int k = 0; k < SV::KL; ++k) {
      const int e = tid + k * NT, r = e / SV::CL, c = e - r * SV::CL;
      sv.vl[k] = CT(0);
      if (r < lnr && c < lnc)
        sv.vl[k] = ldg(pcoef, ((unsigned)sband<false>(lr0 + r, nL) << P_.lgP) +
                                    (unsigned)sband<false>(lc0 + c, nL));
    }
    static_for<2, L + 1>([&](auto lcst) {
      constexpr int l = decltype(lcst)::value;
      constexpr int NUR = fast_nu<LF>(BHp, l), NUC = fast_nu<LF>(BWp, l);
      constexpr int TOT = 3 * NUR * NUC, KS = (TOT + NT - 1) / NT;
      const int n = P_.P >> (l - 1), h = n >> 1;
      const int ur0 = (P_.wr.ca[l] >> 1) - MXLO, nur = ((P_.wr.cb[l] - P_.wr.ca[l]) >> 1) + MXLO + MXHI;
      const int uc0 = (P_.wc.ca[l] >> 1) - MXLO, nuc = ((P_.wc.cb[l] - P_.wc.ca[l]) >> 1) + MXLO + MXHI;
      const bool drop = l <= L - lc;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int e = tid + k * NT;
        const int c = e % NUC, t = e / NUC, r = t % NUR, q = t / NUR;
        sv.vd[l - 2][k] = CT(0);
        if (!drop && e < TOT && r < nur && c < nuc) {
          const int row = q == 0 ? sband<false>(ur0 + r, n) : h + dband<false>(ur0 + r, n);
          const int col = q == 1 ? sband<false>(uc0 + c, n) : h + dband<false>(uc0 + c, n);
          sv.vd[l - 2][k] = ldg(pcoef, ((unsigned)row << P_.lgP) + (unsigned)col);
        }
      }
    });
  };
  auto store_plane = [&](auto pcst, auto& sv) {
    constexpr int p = decltype(pcst)::value;
    constexpr int BHp = p == 0 ? BH : BH / 2, BWp = p == 0 ? BW : BW / 2;
    constexpr int PITCH = p == 0 ? SM::PY : SM::PC;
    using SV = std::remove_reference_t<decltype(sv)>;
    V* llbuf = p == 0 ? sm.BY[0] : sm.BC[p > 0 ? p - 1 : 0][0];
    CT* det = p == 0 ? sm.detY : sm.detC[p > 0 ? p - 1 : 0];
#pragma unroll
    for (int k = 0; k < SV::KL; ++k) {
      const int e = tid + k * NT, r = e / SV::CL, c = e - r * SV::CL;
      if (r < SV::RL) llbuf[r * PITCH + c] = deq(sv.vl[k], qs);
    }
    static_for<2, L + 1>([&](auto lcst) {
      constexpr int l = decltype(lcst)::value;
      constexpr int NUR = fast_nu<LF>(BHp, l), NUC = fast_nu<LF>(BWp, l);
      constexpr int TOT = 3 * NUR * NUC, KS = (TOT + NT - 1) / NT;
      constexpr int OFF = SM::lvl_off(BHp, BWp, l);
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int e = tid + k * NT;
        if (e < TOT) det[OFF + e] = sv.vd[l - 2][k];
      }
    });
  };
  load_plane(std::integral_constant<int, 0>{}, sv0);
  if constexpr (NP == 3) {
    load_plane(std::integral_constant<int, 1>{}, sv1);
    load_plane(std::integral_constant<int, 2>{}, sv2);
  }
  store_plane(std::integral_constant<int, 0>{}, sv0);
  if constexpr (NP == 3) {
    store_plane(std::integral_constant<int, 1>{}, sv1);
    store_plane(std::integral_constant<int, 2>{}, sv2);
  }
  __syncthreads();

  // ---- coarse levels L .. 2 from LDS, all planes per phase
  static_for_down<L, 1>([&](auto lcst) {
    constexpr int l = decltype(lcst)::value;
    constexpr int bi = (L - l) & 1;   // input buffer index at this level
    int start[NP], sh[NP], slots = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const FastGeo<LF, L>& G_ = geo[p > 0 ? 1 : 0];
      const int nr = G_.wr.cb[l] - G_.wr.ca[l], nc = G_.wc.cb[l] - G_.wc.ca[l];
      const int nrun = nr >= 4 ? (nr + 3) >> 2 : 1;
      sh[p] = ceil_log2(nc >> 1);
      start[p] = slots;
      slots += nrun << sh[p];
    }
    for (int i = tid; i < slots; i += NT) {
      auto plane_task = [&](auto pcst) {
        constexpr int p = decltype(pcst)::value;
        constexpr int BHp = p == 0 ? BH : BH / 2, BWp = p == 0 ? BW : BW / 2;
        constexpr int PITCH = p == 0 ? SM::PY : SM::PC;
        constexpr int NUR = fast_nu<LF>(BHp, l), NUC = fast_nu<LF>(BWp, l);
        constexpr int OFF = SM::lvl_off(BHp, BWp, l);
        bool mine = i >= start[p];
        if constexpr (p + 1 < NP) mine = mine && i < start[p + 1];
        if (!mine) return;
        const FastGeo<LF, L>& P_ = geo[p > 0 ? 1 : 0];
        const int car = P_.wr.ca[l], nr = P_.wr.cb[l] - car;
        const int cac = P_.wc.ca[l], nc = P_.wc.cb[l] - cac;
        const int loc = i - start[p], q = loc >> sh[p], j = loc & ((1 << sh[p]) - 1);
        if (2 * j >= nc) return;
        const V* in = p == 0 ? sm.BY[bi] : sm.BC[p > 0 ? p - 1 : 0][bi];
        V* out = p == 0 ? sm.BY[bi ^ 1] : sm.BC[p > 0 ? p - 1 : 0][bi ^ 1];
        const CT* det = (p == 0 ? sm.detY : sm.detC[p > 0 ? p - 1 : 0]) + OFF;
        const int ur0 = (car >> 1) - MXLO, uc0 = (cac >> 1) - MXLO;
        const int m = P_.P >> (l - 1);
        const int cc = cac + 2 * j;
        if (nr >= 4) {
          const int rr = car + min(q * 4, nr - 4);
          staged_task<LF, 4, PITCH, NUR, NUC>(in, P_.wr.wa[l + 1], P_.wc.wa[l + 1], det, ur0, uc0,
                                              qs, rr, cc, out, P_.wr.wa[l], P_.wc.wa[l],
                                              P_.wr.wb[l], P_.wc.wb[l], m);
        } else {
          staged_task<LF, 2, PITCH, NUR, NUC>(in, P_.wr.wa[l + 1], P_.wc.wa[l + 1], det, ur0, uc0,
                                              qs, car, cc, out, P_.wr.wa[l], P_.wc.wa[l],
                                              P_.wr.wb[l], P_.wc.wb[l], m);
        }
      };
      plane_task(std::integral_constant<int, 0>{});
      if constexpr (NP == 3) {
        plane_task(std::integral_constant<int, 1>{});
        plane_task(std::integral_constant<int, 2>{});
      }
    }
    __syncthreads();
  });
  constexpr int bfin = (L - 1) & 1;   // buffer holding W_2

  // ---- finest chroma level (threads split between Cb and Cr), residual, clip
  if constexpr (NP == 3) {
    const V* w2 = pc ? sm.BC[1][bfin] : sm.BC[0][bfin];
    const WV_G CT* ccoef = pc ? coefs[2] : coefs[1];
    if constexpr (WAVE_UNIFORM) ccoef = uniform(ccoef);
    V o[TRC][2];
    level_task<LF, TRC, false, SM::PC>(w2, geo[NG - 1].wr.wa[2], geo[NG - 1].wc.wa[2], ccoef, lgT - 1, T >> 1,
                                      drop1, qs, crr, ccc, o);
    V* chr = sm.CHR + pc * (BH / 2) * (BW / 2);
#pragma unroll
    for (int i = 0; i < TRC; ++i) {
      V b0, b1;
      unpack2(rc[i], b0, b1);
      const V a0 = clip255(o[i][0] + b0), a1 = clip255(o[i][1] + b1);
      store2(at(refC, (unsigned)((crr + i) * (T >> 1) + ccc)), a0, a1);
      chr[(cq2 * TRC + i) * (BW / 2) + 2 * cp2] = a0;
      chr[(cq2 * TRC + i) * (BW / 2) + 2 * cp2 + 1] = a1;
    }
    __syncthreads();
  }

  // ---- finest luma level, residual, clip, colour
  {
    V o[TR][2];
    level_task<LF, TR, false, SM::PY>(sm.BY[bfin], geo[0].wr.wa[2], geo[0].wc.wa[2], coefs[0], lgT,
                                      T, drop1, qs, lrr, lcc, o);
    const bool has_out = (job.flags & kJobHasOut) != 0;
    const unsigned plane = (unsigned)T * T;
    WV_G RT* out = uniform((WV_G RT*)job.out + (size_t)item.slot * NP * plane);
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const unsigned g = (unsigned)((lrr + i) * T + lcc);
      V b0, b1;
      unpack2(ry[i], b0, b1);
      const V y0 = clip255(o[i][0] + b0), y1 = clip255(o[i][1] + b1);
      store2(at(refY, g), y0, y1);
      if (has_out) {
        if constexpr (NP == 3) {
          const int ci = ((lq * TR + i) >> 1) * (BW / 2) + lp;
          const V cb = sm.CHR[ci], cr = sm.CHR[(BH / 2) * (BW / 2) + ci];
          V R0, G0, B0, R1, G1, B1;
          to_rgb(y0, cb, cr, R0, G0, B0);
          to_rgb(y1, cb, cr, R1, G1, B1);
          store2(at(out, g), R0, R1);
          store2(at(out, g + plane), G0, G1);
          store2(at(out, g + 2u * plane), B0, B1);
        } else {
          store2(at(out, g), y0, y1);
        }
      }
    }
  }
  __syncthreads();
}

template <class LF, int FMT, int BW, int BH, int TR, int L, bool PERSIST>
__global__ __launch_bounds__((BW / 2) * (BH / TR)) void k_fused_fast(const WorkArgs a) {
  __shared__ FastSmem<LF, FMT, BW, BH, L> sm;
  const int total = a.total_dev ? *a.total_dev : a.total;
  if (!PERSIST) {
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    if (u < total) fast_unit<LF, FMT, BW, BH, TR, L>(sm, a, u);
    return;
  }
  __shared__ int s_unit;
  for (;;) {
    if (threadIdx.x == 0) s_unit = (int)atomicAdd(&a.counter[0], 1u);
    __syncthreads();
    const int u = s_unit;
    __syncthreads();
    if (u >= total) break;
    fast_unit<LF, FMT, BW, BH, TR, L>(sm, a, u);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned done = atomicAdd(&a.counter[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&a.counter[0], 0u);
      atomicExch(&a.counter[1], 0u);
    }
  }
}

}  // namespace wv
