// Device pieces shared by the fused decode kernels (general and fast forms).
#pragma once

#include <type_traits>

#include "wv_dev.h"
#include "wv_internal.h"

namespace wv {

// Upper bound of the layout window W_{k+1} given W_k's length bound w.
template <class LF>
constexpr int wnext(int w) {
  const int n = w / 2 + LF::S_LO + LF::S_HI + 2;
  return n + (n & 1);
}
template <class LF>
constexpr int w_at(int B, int k) {
  int w = B;
  for (int j = 1; j < k; ++j) w = wnext<LF>(w);
  return w;
}
template <class LF>
constexpr int w_max_from(int B, int k) {
  int w = w_at<LF>(B, k), m = 0;
  for (int j = 0; j < 16; ++j) {
    m = w > m ? w : m;
    w = wnext<LF>(w);
  }
  return m;
}

__device__ __forceinline__ int ceil_log2(int x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

// Global-memory pointers: the job table holds generic pointers, and without
// this qualifier every access would compile to FLAT instructions with 64-bit
// per-lane address arithmetic.
#define WV_G __attribute__((address_space(1)))

// A pointer that is the same for the whole group, moved to scalar registers
// so that loads use a scalar base plus a 32-bit vector offset.
template <class T>
__device__ __forceinline__ T* uniform(T* p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// Element at a 32-bit index from a scalar base: the byte offset is formed in
// 32 bits so the access can use the scalar-base + 32-bit-offset form.
template <class T>
__device__ __forceinline__ T ldg(const WV_G T* base, unsigned idx) {
  return *(const WV_G T*)((const WV_G char*)base + idx * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ WV_G T* at(WV_G T* base, unsigned idx) {
  return (WV_G T*)((WV_G char*)base + idx * (unsigned)sizeof(T));
}

// Symmetric-extension index.  Windows reach at most a few samples beyond a
// region, so for regions of 16 or more samples one reflection suffices and is
// branch-free: min(|j|, 2n-2-|j|); smaller regions use the general loop.
// GEN selects the general loop (variants used when some region is smaller).
template <bool GEN>
__device__ __forceinline__ int ext(int j, int n) {
  if (GEN) return wss(j, n);
  const int a = abs(j);
  return min(a, 2 * n - 2 - a);
}
template <bool GEN>
__device__ __forceinline__ int sband(int i, int n) { return ext<GEN>(2 * i, n) >> 1; }
template <bool GEN>
__device__ __forceinline__ int dband(int i, int n) { return ext<GEN>(2 * i + 1, n) >> 1; }

template <class LF, int FMT, int BW, int BH>
struct FusedSmem {
  using V = typename LF::V;
  // ping-pong window buffers per plane, bounded by the level-2 layout window
  // pitches: multiples of 4 (rows are read along columns by consecutive
  // lanes, so no padding against bank conflicts is needed)
  static constexpr int RY = w_max_from<LF>(BH, 2), CY = w_max_from<LF>(BW, 2), PY = (CY + 3) & ~3;
  static constexpr int RC = w_max_from<LF>(BH / 2, 2), CC = w_max_from<LF>(BW / 2, 2),
                       PC = (CC + 3) & ~3;
  static constexpr int NCP = FMT == WV_YUV420 ? 2 : 0;   // chroma planes
  V BY[2][RY * PY];
  V BC[NCP > 0 ? NCP : 1][2][NCP > 0 ? RC * PC : 1];
  V CHR[NCP > 0 ? NCP * (BH / 2) * (BW / 2) : 1];        // reconstructed chroma block
};

// Per-plane state of one block, uniform across the group.
template <class CT, class V>
struct PlaneState {
  const WV_G CT* coef;   // tile-plane coefficients
  int P;            // plane tile edge
  int lgP;          // log2(P)
  int r0, c0, bh, bw;
  V* in;            // window buffer holding the current approximation input
  V* out;           // the other buffer (next level's output)
  int pitch;
};

// One task of level l: output columns cc, cc+1 and rows rr .. rr+TRL of the
// level's region (edge n).  The approximation input is read from the LDS
// window `ll` (pitch pll, origin llr/llc); the details straight from the
// coefficient store (all loads issued before use).
template <class LF, int TRL, bool GEN, int PLL, class CT>
__device__ __forceinline__ void level_task(const typename LF::V* __restrict__ ll, int llr,
                                           int llc, const WV_G CT* __restrict__ coef, int lgP, int n,
                                           bool drop, int qstep, int rr, int cc,
                                           typename LF::V (&out)[TRL][2]) {
  using V = typename LF::V;
  constexpr int NPR = TRL / 2;
  constexpr int NSV = NPR + LF::S_LO + LF::S_HI, NDV = NPR + LF::D_LO + LF::D_HI;
  constexpr int NSH = 1 + LF::S_LO + LF::S_HI, NDH = 1 + LF::D_LO + LF::D_HI;
  const int h = n >> 1;
  const int sr0 = (rr >> 1) - LF::S_LO, dr0 = (rr >> 1) - LF::D_LO;
  const int sc0 = (cc >> 1) - LF::S_LO, dc0 = (cc >> 1) - LF::D_LO;
  int scol[NSH], dcol[NDH];
#pragma unroll
  for (int j = 0; j < NSH; ++j) scol[j] = sband<GEN>(sc0 + j, n);
#pragma unroll
  for (int j = 0; j < NDH; ++j) dcol[j] = h + dband<GEN>(dc0 + j, n);
  // detail loads first
  CT hl[NSV][NDH], lh[NDV][NSH], hh[NDV][NDH];
  if (!drop) {
    // unsigned 32-bit element offsets from a scalar base: global loads with
    // saddr + voffset, no 64-bit per-lane address arithmetic
#pragma unroll
    for (int i = 0; i < NSV; ++i) {
      const unsigned roff = (unsigned)sband<GEN>(sr0 + i, n) << lgP;
#pragma unroll
      for (int j = 0; j < NDH; ++j) hl[i][j] = ldg(coef, roff + (unsigned)dcol[j]);
    }
#pragma unroll
    for (int i = 0; i < NDV; ++i) {
      const unsigned roff = (unsigned)(h + dband<GEN>(dr0 + i, n)) << lgP;
#pragma unroll
      for (int j = 0; j < NSH; ++j) lh[i][j] = ldg(coef, roff + (unsigned)scol[j]);
#pragma unroll
      for (int j = 0; j < NDH; ++j) hh[i][j] = ldg(coef, roff + (unsigned)dcol[j]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < NSV; ++i)
#pragma unroll
      for (int j = 0; j < NDH; ++j) hl[i][j] = CT(0);
#pragma unroll
    for (int i = 0; i < NDV; ++i) {
#pragma unroll
      for (int j = 0; j < NSH; ++j) lh[i][j] = CT(0);
#pragma unroll
      for (int j = 0; j < NDH; ++j) hh[i][j] = CT(0);
    }
  }
  V top[NSV][2], bot[NDV][2];
#pragma unroll
  for (int i = 0; i < NSV; ++i) {
    V s[NSH], d[NDH], x[2];
    const V* lp = ll + (sr0 + i - llr) * PLL + (sc0 - llc);
#pragma unroll
    for (int j = 0; j < NSH; ++j) s[j] = lp[j];
#pragma unroll
    for (int j = 0; j < NDH; ++j) d[j] = deq(hl[i][j], qstep);
    LF::template run<1>(s, d, x);
    top[i][0] = x[0];
    top[i][1] = x[1];
  }
#pragma unroll
  for (int i = 0; i < NDV; ++i) {
    V s[NSH], d[NDH], x[2];
#pragma unroll
    for (int j = 0; j < NSH; ++j) s[j] = deq(lh[i][j], qstep);
#pragma unroll
    for (int j = 0; j < NDH; ++j) d[j] = deq(hh[i][j], qstep);
    LF::template run<1>(s, d, x);
    bot[i][0] = x[0];
    bot[i][1] = x[1];
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
    for (int i = 0; i < TRL; ++i) out[i][c] = x[i];
  }
}

// Two horizontally adjacent reference/output samples.
__device__ __forceinline__ void load2(const WV_G uint8_t* p, int& a, int& b) {
  const uint16_t v = *(const WV_G uint16_t*)p;
  a = v & 0xff;
  b = v >> 8;
}
__device__ __forceinline__ void load2(const WV_G float* p, float& a, float& b) {
  a = p[0];
  b = p[1];
}
__device__ __forceinline__ void store2(WV_G uint8_t* p, int a, int b) {
  *(WV_G uint16_t*)p = (uint16_t)(a | (b << 8));
}
__device__ __forceinline__ void store2(WV_G float* p, float a, float b) {
  p[0] = a;
  p[1] = b;
}


// Compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
// Descending: I = B, B-1, .. E+1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for_down(F&& f) {
  if constexpr (B > E) {
    f(std::integral_constant<int, B>{});
    static_for_down<B - 1, E>(f);
  }
}

}  // namespace wv
