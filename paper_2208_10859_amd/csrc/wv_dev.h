// Device helpers shared by the fused, plain and encoder kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// q is an int16 index and step <= 65535: both fit the 24-bit multiplier.
__device__ __forceinline__ int deq(int16_t q, int step) { return __mul24((int)q, step); }
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


}  // namespace wv
