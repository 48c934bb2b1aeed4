// Row-strip fused decode (Section 3.1's viewport decode, every step in one
// launch).  One work unit is one visible tile and a strip of R luma rows
// (R/2 rows of each chroma plane) across the whole tile width.
//
// Each row of a level is spread over consecutive lanes, every lane owning C
// adjacent output columns (C/2 low- and C/2 high-band samples), so the
// horizontal lifting needs only one value from each neighbouring lane per
// lifting step (a DPP lane shift); the tile's left and right edges are the
// first and last lane of a row, where whole-sample symmetric extension keeps
// the lane's own value.  The vertical lifting streams down the rows inside
// each lane: a handful of rows of state, outputs emitted pair by pair.
// Rows are the same for every lane of a wave, so row indices, the symmetric
// extension of rows and row addresses are scalar work, and loads are a
// scalar row base plus a fixed per-lane offset.
//
// The coarse levels of the strip's dependency cone are computed into LDS
// windows (full width, the rows the next finer level reads); the finest
// chroma rows go to LDS too, and the finest luma rows are combined with them
// for the colour conversion.  Phases (one barrier each): chroma level L,
// then luma level l+1 with chroma level l for l = L-1 .. 1, then luma level 1.
#pragma once

#include "wv_fused_common.h"

namespace wv {
namespace strip {

// Clang vector types: unlike the HIP vector structs they load and store
// through address-space-qualified pointers.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Lane layout of a level whose rows hold N output samples.
template <int N>
struct RL {
  static constexpr int C = N >= 128 ? N / 64 : 2;   // output columns per lane
  static constexpr int H = C / 2;                   // low (and high) band samples per lane
  static constexpr int G = N / C;                   // lanes per row
  static constexpr int S = 64 / G;                  // rows side by side in one wave
};

// Value of the same register in the previous / next lane of the wave; the
// first / last lane of a row gets `edge` instead.
template <int G>
__device__ __forceinline__ int from_left(int edge, int v, int g) {
  int r = __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false);   // wave_shr:1
  if constexpr (G < 64) r = g == 0 ? edge : r;
  return r;
}
template <int G>
__device__ __forceinline__ int from_right(int edge, int v, int g) {
  int r = __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xf, 0xf, false);   // wave_shl:1
  if constexpr (G < 64) r = g == G - 1 ? edge : r;
  return r;
}
template <int G>
__device__ __forceinline__ float from_left(float edge, float v, int g) {
  return __int_as_float(from_left<G>(__float_as_int(edge), __float_as_int(v), g));
}
template <int G>
__device__ __forceinline__ float from_right(float edge, float v, int g) {
  return __int_as_float(from_right<G>(__float_as_int(edge), __float_as_int(v), g));
}

// One row of a level: C outputs per lane from H low-band values s and H
// high-band values d (the same lifting as the 1D definitions; the
// neighbouring lanes supply the samples just outside the lane's range).
template <class LF, int N>
struct HLift;

template <int N>
struct HLift<Inv53, N> {
  static constexpr int H = RL<N>::H, G = RL<N>::G;
  __device__ static __forceinline__ void run(const int (&s)[H], const int (&d)[H], int g,
                                             int (&x)[2 * H]) {
    const int dl = from_left<G>(d[0], d[H - 1], g);   // d[-1] = d[0] at the left edge
    int e[H];
#pragma unroll
    for (int k = 0; k < H; ++k) e[k] = s[k] - (((k ? d[k - 1] : dl) + d[k] + 2) >> 2);
    const int er = from_right<G>(e[H - 1], e[0], g);  // x[2M] = x[2M-2] at the right edge
#pragma unroll
    for (int k = 0; k < H; ++k) {
      x[2 * k] = e[k];
      x[2 * k + 1] = d[k] + ((e[k] + (k + 1 < H ? e[k + 1] : er)) >> 1);
    }
  }
};

template <int N>
struct HLift<Inv97, N> {
  static constexpr int H = RL<N>::H, G = RL<N>::G;
  __device__ static __forceinline__ void run(const float (&s)[H], const float (&d)[H], int g,
                                             float (&x)[2 * H]) {
    const float K = (float)WV_K97, IK = (float)(1.0 / WV_K97);
    const float A = (float)WV_A97, B = (float)WV_B97, Gm = (float)WV_G97, D = (float)WV_D97;
    float e[H], o[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
      o[k] = d[k] * IK;
      e[k] = K * s[k];
    }
    {
      const float l = from_left<G>(o[0], o[H - 1], g);
#pragma unroll
      for (int k = 0; k < H; ++k) e[k] = e[k] - D * ((k ? o[k - 1] : l) + o[k]);
    }
    {
      const float r = from_right<G>(e[H - 1], e[0], g);
#pragma unroll
      for (int k = 0; k < H; ++k) o[k] = o[k] - Gm * (e[k] + (k + 1 < H ? e[k + 1] : r));
    }
    {
      const float l = from_left<G>(o[0], o[H - 1], g);
#pragma unroll
      for (int k = 0; k < H; ++k) e[k] = e[k] - B * ((k ? o[k - 1] : l) + o[k]);
    }
    {
      const float r = from_right<G>(e[H - 1], e[0], g);
#pragma unroll
      for (int k = 0; k < H; ++k) o[k] = o[k] - A * (e[k] + (k + 1 < H ? e[k + 1] : r));
    }
#pragma unroll
    for (int k = 0; k < H; ++k) {
      x[2 * k] = e[k];
      x[2 * k + 1] = o[k];
    }
  }
};

// Vertical lifting streamed down the rows.  Push I carries the horizontally
// reconstructed low-band row t and high-band row t of the level, for
// t = j0 - D_LO + I; output pair j0 + I - LAG (rows 2j, 2j+1) is emitted once
// its inputs are in.
template <class LF, int C>
struct VStream;

template <int C>
struct VStream<Inv53, C> {
  static constexpr int LAG = 2;
  int bp[C], ep[C];   // high row t-1, even output row 2t-2
  template <int I, class Emit>
  __device__ __forceinline__ void push(const int (&top)[C], const int (&bot)[C], Emit& emit) {
    if constexpr (I == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) bp[c] = bot[c];
    } else {
      int e[C];
#pragma unroll
      for (int c = 0; c < C; ++c) e[c] = top[c] - ((bp[c] + bot[c] + 2) >> 2);
      if constexpr (I >= 2) {
        int o[C];
#pragma unroll
        for (int c = 0; c < C; ++c) o[c] = bp[c] + ((ep[c] + e[c]) >> 1);
        emit.template pair<I - LAG>(ep, o);
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        ep[c] = e[c];
        bp[c] = bot[c];
      }
    }
  }
};

template <int C>
struct VStream<Inv97, C> {
  static constexpr int LAG = 4;
  float o0p[C], e1p[C], o1p[C], e2p[C];
  template <int I, class Emit>
  __device__ __forceinline__ void push(const float (&top)[C], const float (&bot)[C], Emit& emit) {
    const float K = (float)WV_K97, IK = (float)(1.0 / WV_K97);
    const float A = (float)WV_A97, B = (float)WV_B97, Gm = (float)WV_G97, D = (float)WV_D97;
    float o0[C];
#pragma unroll
    for (int c = 0; c < C; ++c) o0[c] = bot[c] * IK;
    if constexpr (I >= 1) {
      float e1[C], o1[C], e2[C];
#pragma unroll
      for (int c = 0; c < C; ++c) e1[c] = K * top[c] - D * (o0p[c] + o0[c]);
      if constexpr (I >= 2) {
#pragma unroll
        for (int c = 0; c < C; ++c) o1[c] = o0p[c] - Gm * (e1p[c] + e1[c]);
      }
      if constexpr (I >= 3) {
#pragma unroll
        for (int c = 0; c < C; ++c) e2[c] = e1p[c] - B * (o1p[c] + o1[c]);
      }
      if constexpr (I >= 4) {
        float o2[C];
#pragma unroll
        for (int c = 0; c < C; ++c) o2[c] = o1p[c] - A * (e2p[c] + e2[c]);
        emit.template pair<I - LAG>(e2p, o2);
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if constexpr (I >= 3) e2p[c] = e2[c];
        if constexpr (I >= 2) o1p[c] = o1[c];
        e1p[c] = e1[c];
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) o0p[c] = o0[c];
  }
};

// ------------------------------------------------------------ small vectors
// H consecutive coefficients (int16 dequantised, or float) from global memory.
template <int H>
__device__ __forceinline__ void ld_coef(const WV_G int16_t* p, int q, int (&v)[H]) {
  if constexpr (H == 4) {
    const u32x2 w = *(const WV_G u32x2*)p;
    v[0] = __mul24((int)(int16_t)(w.x & 0xffffu), q);
    v[1] = __mul24((int)w.x >> 16, q);
    v[2] = __mul24((int)(int16_t)(w.y & 0xffffu), q);
    v[3] = __mul24((int)w.y >> 16, q);
  } else if constexpr (H == 2) {
    const uint32_t w = *(const WV_G uint32_t*)p;
    v[0] = __mul24((int)(int16_t)(w & 0xffffu), q);
    v[1] = __mul24((int)w >> 16, q);
  } else {
    static_assert(H == 1, "lane width");
    v[0] = __mul24((int)*p, q);
  }
}
template <int H>
__device__ __forceinline__ void ld_coef(const WV_G float* p, int, float (&v)[H]) {
  if constexpr (H == 4) {
    const f32x4 w = *(const WV_G f32x4*)p;
    v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
  } else if constexpr (H == 2) {
    const f32x2 w = *(const WV_G f32x2*)p;
    v[0] = w.x; v[1] = w.y;
  } else {
    v[0] = *p;
  }
}

// N consecutive LDS values.
template <int N, class V>
__device__ __forceinline__ void ld_lds(const V* p, V (&v)[N]) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (int k = 0; k < N; k += 4) {
      const int4 w = *(const int4*)(p + k);
      v[k] = __builtin_bit_cast(V, w.x); v[k + 1] = __builtin_bit_cast(V, w.y);
      v[k + 2] = __builtin_bit_cast(V, w.z); v[k + 3] = __builtin_bit_cast(V, w.w);
    }
  } else if constexpr (N == 2) {
    const int2 w = *(const int2*)p;
    v[0] = __builtin_bit_cast(V, w.x); v[1] = __builtin_bit_cast(V, w.y);
  } else {
    v[0] = p[0];
  }
}
template <int N, class V>
__device__ __forceinline__ void st_lds(V* p, const V (&v)[N]) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (int k = 0; k < N; k += 4)
      *(int4*)(p + k) = make_int4(__builtin_bit_cast(int, v[k]), __builtin_bit_cast(int, v[k + 1]),
                                  __builtin_bit_cast(int, v[k + 2]), __builtin_bit_cast(int, v[k + 3]));
  } else if constexpr (N == 2) {
    *(int2*)p = make_int2(__builtin_bit_cast(int, v[0]), __builtin_bit_cast(int, v[1]));
  } else {
    p[0] = v[0];
  }
}

// N samples of a plane row: uint8 (5/3) or float (9/7).
template <int N>
__device__ __forceinline__ void ld_px(const WV_G uint8_t* p, int (&v)[N]) {
  if constexpr (N == 8) {
    const u32x2 w = *(const WV_G u32x2*)p;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = (w.x >> (8 * k)) & 0xff;
      v[4 + k] = (w.y >> (8 * k)) & 0xff;
    }
  } else if constexpr (N == 4) {
    const uint32_t w = *(const WV_G uint32_t*)p;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (w >> (8 * k)) & 0xff;
  } else {
    static_assert(N == 2, "row width");
    const uint32_t w = *(const WV_G uint16_t*)p;
    v[0] = w & 0xff;
    v[1] = w >> 8;
  }
}
template <int N>
__device__ __forceinline__ void ld_px(const WV_G float* p, float (&v)[N]) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (int k = 0; k < N; k += 4) {
      const f32x4 w = *(const WV_G f32x4*)(p + k);
      v[k] = w.x; v[k + 1] = w.y; v[k + 2] = w.z; v[k + 3] = w.w;
    }
  } else {
    const f32x2 w = *(const WV_G f32x2*)p;
    v[0] = w.x; v[1] = w.y;
  }
}

// Prefetched reference rows of a segment (up to 8 pairs).  8-bit samples stay
// packed as loaded (a quarter of the registers) and are taken apart where
// they are added; float samples are kept as they are.
template <class RT, int C>
struct RefRows;
template <int C>
struct RefRows<uint8_t, C> {
  static constexpr int W = (C + 3) / 4;
  uint32_t w[2 * 8][W];
  // intra frames: nothing to add
  template <int K>
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int r = 0; r < 2 * K; ++r)
#pragma unroll
      for (int k = 0; k < W; ++k) w[r][k] = 0u;
  }
  __device__ __forceinline__ void load(int row, const WV_G uint8_t* p) {
    if constexpr (C == 8) {
      const u32x2 v = *(const WV_G u32x2*)p;
      w[row][0] = v.x;
      w[row][1] = v.y;
    } else if constexpr (C == 4) {
      w[row][0] = *(const WV_G uint32_t*)p;
    } else {
      static_assert(C == 2, "row width");
      w[row][0] = *(const WV_G uint16_t*)p;
    }
  }
  // the row from LDS (the strip's chroma rows of the previous frame)
  __device__ __forceinline__ void load_lds(int row, const uint8_t* p) {
    if constexpr (C == 8) {
      const uint2 v = *(const uint2*)p;
      w[row][0] = v.x;
      w[row][1] = v.y;
    } else if constexpr (C == 4) {
      w[row][0] = *(const uint32_t*)p;
    } else {
      w[row][0] = *(const uint16_t*)p;
    }
  }
  __device__ __forceinline__ void set(int row, int k, uint32_t v) { w[row][k] = v; }
  __device__ __forceinline__ int get(int row, int c) const { return (w[row][c >> 2] >> (8 * (c & 3))) & 0xff; }
};
template <int C>
struct RefRows<float, C> {
  float v[2 * 8][C];
  template <int K>
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int r = 0; r < 2 * K; ++r)
#pragma unroll
      for (int k = 0; k < C; ++k) v[r][k] = 0.0f;
  }
  __device__ __forceinline__ void load(int row, const WV_G float* p) { ld_px<C>(p, v[row]); }
  __device__ __forceinline__ void load_lds(int row, const float* p) { ld_lds<C>(p, v[row]); }
  __device__ __forceinline__ float get(int row, int c) const { return v[row][c]; }
};

// Byte permutation (V_PERM_B32): byte i of the result is byte sel_i of the
// eight bytes {lo (0..3), hi (4..7)}; selector 0x0c gives 0x00, 0x0d 0xff.
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}
// Byte packing of values already clipped to 0..255, as byte permutations.
// Packing with shifts and ORs let instruction selection fold a preceding
// shift and clamp of two values into V_ASHR_PK_U8_I32, which writes only the
// low half of its destination, while the code this toolchain generated after
// it ORed further bytes into the upper half as if it were zero: the
// register's stale bytes reached the output (clipped odd rows of the 5/3
// inverse, (a + b) >> 1 with no residual).  A permutation of whole registers
// offers no such pattern.
__device__ __forceinline__ uint32_t pack4(int a, int b, int c, int d) {
  const uint32_t ab = perm((uint32_t)b, (uint32_t)a, 0x0c0c0400u);   // a0 b0 0 0
  const uint32_t cd = perm((uint32_t)d, (uint32_t)c, 0x0c0c0400u);   // c0 d0 0 0
  return perm(cd, ab, 0x05040100u);                                   // a0 b0 c0 d0
}
__device__ __forceinline__ uint16_t pack2(int a, int b) {
  return (uint16_t)perm((uint32_t)b, (uint32_t)a, 0x0c0c0400u);
}

// 8-bit colour conversion on pairs of 16-bit halves.  A luma sample y is held
// as 0xff00 + y; a colour term t (the Q16 JFIF term of one chroma sample,
// |t| < 256) as B = 0xff00 - t in both halves.  Then
//   sat_sub_u16(0xff00 + y, B) = max(y + t, 0)
//   sat_add_u16(that, 0xff00) = 0xff00 + min(max(y + t, 0), 255),
// so the low byte of each half is clip(y + t, 0, 255).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
// halves 0xff00 + a, 0xff00 + b from the low bytes of a and b
__device__ __forceinline__ uint32_t ypair(int a, int b) {
  return perm((uint32_t)b, (uint32_t)a, 0x0d040d00u);
}
// bytes 0 and 2 of lo, then bytes 0 and 2 of hi
__device__ __forceinline__ uint32_t low_bytes(uint32_t lo, uint32_t hi) {
  return perm(hi, lo, 0x06040200u);
}
__device__ __forceinline__ uint32_t clip_add(uint32_t yp, uint32_t b2) {
  u16x2 r = __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, yp), __builtin_bit_cast(u16x2, b2));
  r = __builtin_elementwise_add_sat(r, (u16x2){0xff00, 0xff00});
  return __builtin_bit_cast(uint32_t, r);
}
// B = 0xff00 - t in both halves, for t = (k * c' + 32768) >> 16 (c' = c - 128
// a chroma offset, k one of the Q16 factors, or the sum of two such
// products): -floor(v / 2^16) = floor((2^16 - 1 - v) / 2^16), so
// B = (0xff000000 + 32767 - k * c') >> 16, whose 32-bit value lies inside
// [0, 2^32) for every 8-bit chroma pair.  w is that 32-bit value.
__device__ __forceinline__ uint32_t term2(uint32_t w) { return perm(w, w, 0x03020302u); }
constexpr uint32_t kTermBias = 0xff000000u + 32767u;
template <int N>
__device__ __forceinline__ void st_px(WV_G uint8_t* p, const int (&v)[N]) {
  if constexpr (N == 8) {
    *(WV_G u32x2*)p = u32x2{pack4(v[0], v[1], v[2], v[3]), pack4(v[4], v[5], v[6], v[7])};
  } else if constexpr (N == 4) {
    *(WV_G uint32_t*)p = pack4(v[0], v[1], v[2], v[3]);
  } else {
    *(WV_G uint16_t*)p = pack2(v[0], v[1]);
  }
}
template <int N>
__device__ __forceinline__ void st_px(WV_G float* p, const float (&v)[N]) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (int k = 0; k < N; k += 4) *(WV_G f32x4*)(p + k) = f32x4{v[k], v[k + 1], v[k + 2], v[k + 3]};
  } else {
    *(WV_G f32x2*)p = f32x2{v[0], v[1]};
  }
}

// ------------------------------------------------------------ geometry
// Rows the strip's cone needs at every level (output rows of level l:
// [a[l], b[l])), even-aligned.  Level l reads low-band rows
// [a/2 - S_LO, b/2 + S_HI) of level l+1's output, symmetric-extended.
template <class LF, int L>
__device__ __forceinline__ void cone(int r0, int rows, int P, int (&a)[L + 1], int (&b)[L + 1]) {
  a[1] = r0;
  b[1] = r0 + rows;
#pragma unroll
  for (int l = 1; l < L; ++l) {
    const int M = P >> l;
    const int u = (a[l] >> 1) - LF::S_LO, v = (b[l] >> 1) + LF::S_HI;
    int lo = max(u, 0), hi = min(v, M);
    if (u < 0) hi = max(hi, 1 - u);         // s[-i] = s[i]
    if (v > M) lo = min(lo, 2 * M - v);     // s[M+i] = s[M-1-i]
    a[l + 1] = lo & ~1;
    b[l + 1] = min((hi + 1) & ~1, M);
  }
}

// Compile-time bound of the rows of level l's window for a strip of `rows`.
template <class LF>
constexpr int win_rows(int rows, int P, int l) {
  int w = rows;
  for (int k = 1; k < l; ++k) {
    int nxt = w / 2 + LF::S_LO + LF::S_HI + 2;
    nxt += nxt & 1;
    const int m = P >> k;
    w = nxt < m ? nxt : m;
  }
  return w;
}
template <class LF>
constexpr int win_elems(int rows, int P, int L, int parity) {
  int m = 1;
  for (int l = 2; l <= L; ++l)
    if ((l & 1) == parity) {
      const int e = win_rows<LF>(rows, P, l) * (P >> (l - 1));
      m = e > m ? e : m;
    }
  return m;
}

// Symmetric extension of a row index of a level of n rows (band index t of
// the low band: 2t, of the high band: 2t+1).
template <int N>
__device__ __forceinline__ int ext_row(int j) {
  if constexpr (N >= 8) {
    const int a = abs(j);
    return min(a, 2 * N - 2 - a);
  } else {
    return wss(j, N);
  }
}

// Largest window of the even levels from 4 up (level 2's is the largest).
template <class LF>
constexpr int win_elems_from4(int rows, int P, int L) {
  int m = 0;
  for (int l = 4; l <= L; l += 2) {
    const int e = win_rows<LF>(rows, P, l) * (P >> (l - 1));
    m = e > m ? e : m;
  }
  return m;
}

// LDS of one unit.  Phased schedule: a window per parity and plane.  Chain
// schedule (YUV420): the chroma odd-level windows live inside the luma
// even-level window, after its level-4 rows -- they are dead by the time luma
// level 2 fills that window (the chains of every plane end before it), and
// luma level 4 and the chroma chains run at the same time on other rows.
template <class LF, int FMT, int P, int L, int R, int SCHED>
struct Smem {
  using V = typename LF::V;
  using RT = typename CoefT<LF>::R;
  static constexpr int NC = FMT == WV_YUV420 ? 2 : 0;
  static constexpr bool ALIAS = NC && SCHED == 1;
  static constexpr int YB = win_elems<LF>(R, P, L, 1);
  static constexpr int CA = NC ? win_elems<LF>(R / 2, P / 2, L, 0) : 1;
  static constexpr int CB = NC ? win_elems<LF>(R / 2, P / 2, L, 1) : 1;
  static constexpr int Y4 = (win_elems_from4<LF>(R, P, L) + 3) & ~3;   // keeps cb 16-byte aligned
  static constexpr int YA0 = win_elems<LF>(R, P, L, 0);
  static constexpr int YA = ALIAS ? (YA0 > Y4 + NC * CB ? YA0 : Y4 + NC * CB) : YA0;
  static constexpr int CBS = ALIAS ? 1 : CB;                            // separate cb storage
  static constexpr int CHR = NC ? (R / 2) * (P / 2) : 4;
  static_assert(!ALIAS || CB % 4 == 0, "chroma windows keep 16-byte alignment");
  alignas(16) V ya_[YA];
  alignas(16) V yb[YB];
  alignas(16) V ca[NC ? NC : 1][CA];
  alignas(16) V cb_[NC ? NC : 1][CBS];
  alignas(16) RT chr[NC ? NC : 1][CHR];   // finest chroma rows of the strip
  __device__ __forceinline__ V* ya() { return ya_; }
  __device__ __forceinline__ V* cb(int p) { return ALIAS ? ya_ + Y4 + p * CB : cb_[p]; }
};

// Chroma samples in LDS: bytes (5/3) or floats (9/7).
template <int N>
__device__ __forceinline__ void st_chr(uint8_t* p, const int (&v)[N]) {
  if constexpr (N == 8) {
    *(uint2*)p = make_uint2(pack4(v[0], v[1], v[2], v[3]), pack4(v[4], v[5], v[6], v[7]));
  } else if constexpr (N == 4) {
    *(uint32_t*)p = pack4(v[0], v[1], v[2], v[3]);
  } else {
    *(uint16_t*)p = pack2(v[0], v[1]);
  }
}
template <int N>
__device__ __forceinline__ void st_chr(float* p, const float (&v)[N]) {
  st_lds<N>(p, v);
}
template <int N>
__device__ __forceinline__ void ld_chr(const uint8_t* p, int (&v)[N]) {
  if constexpr (N == 4) {
    const uint32_t w = *(const uint32_t*)p;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (w >> (8 * k)) & 0xff;
  } else if constexpr (N == 2) {
    const uint32_t w = *(const uint16_t*)p;
    v[0] = w & 0xff;
    v[1] = w >> 8;
  } else {
    v[0] = *p;
  }
}
template <int N>
__device__ __forceinline__ void ld_chr(const float* p, float (&v)[N]) {
  ld_lds<N>(p, v);
}

// Per-plane state of one work unit (uniform).
template <class LF, int L, class SRC = const WV_G typename CoefT<LF>::T*>
struct Plane {
  using CT = typename CoefT<LF>::T;
  using RT = typename CoefT<LF>::R;
  SRC coef;                  // the stored coefficients, or an inter-frame set's bands
  WV_G RT* ref;
  typename LF::V* win[2];    // LDS windows (even / odd levels)
  int a[L + 1], b[L + 1];
};

// Emitters: where a level's output rows go.
// Coarse level: into the level's LDS window.
template <class V, int N, int C>
struct ToWindow {
  V* base;       // window origin of this lane's columns
  int j0, kk, a;
  template <int J>
  __device__ __forceinline__ void pair(const V (&xe)[C], const V (&xo)[C]) {
    if (J < kk) {
      V* p = base + (2 * (j0 + J) - a) * N;
      st_lds<C>(p, xe);
      st_lds<C>(p + N, xo);
    }
  }
};

// Finest chroma rows: residual, clip, new reference (WREF), and the strip's
// chroma rows for the colour conversion.
template <class LF, int N, int C, bool WREF = true>
struct ChromaOut {
  using V = typename LF::V;
  using RT = typename CoefT<LF>::R;
  WV_G RT* ref;   // row 0 of the tile's plane (uniform)
  unsigned lo;    // this lane's first column
  RT* chr;        // this lane's columns of strip row 0
  int j0, r0;
  bool wref;      // store the new reference rows to memory
  RefRows<RT, C> refv;   // prefetched reference rows (zero for intra frames)
  template <int J>
  __device__ __forceinline__ void pair(const V (&xe)[C], const V (&xo)[C]) {
    const int r = 2 * (j0 + J);
    V ye[C], yo[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      ye[c] = clip255(xe[c] + refv.get(2 * J, c));
      yo[c] = clip255(xo[c] + refv.get(2 * J + 1, c));
    }
    if constexpr (sizeof(RT) == 1 && C == 4) {
      // one packed word per row, stored to the reference and to LDS
      const uint32_t we = pack4(ye[0], ye[1], ye[2], ye[3]);
      const uint32_t wo = pack4(yo[0], yo[1], yo[2], yo[3]);
      if constexpr (WREF) {
        if (wref) {
          *(WV_G uint32_t*)at(ref + r * N, lo) = we;
          *(WV_G uint32_t*)at(ref + (r + 1) * N, lo) = wo;
        }
      }
      *(uint32_t*)(chr + (r - r0) * N) = we;
      *(uint32_t*)(chr + (r + 1 - r0) * N) = wo;
      return;
    }
    if constexpr (WREF) {
      if (wref) {
        st_px<C>(at(ref + r * N, lo), ye);
        st_px<C>(at(ref + (r + 1) * N, lo), yo);
      }
    }
    st_chr<C>(chr + (r - r0) * N, ye);
    st_chr<C>(chr + (r + 1 - r0) * N, yo);
  }
};

// Finest luma rows: residual, clip, new reference (WREF), colour conversion
// with the strip's chroma rows, output.
template <class LF, int FMT, int N, int C, bool WREF = true>
struct LumaOut {
  using V = typename LF::V;
  using RT = typename CoefT<LF>::R;
  WV_G RT* ref;       // row 0 of the tile's plane (uniform)
  WV_G RT* out;       // row 0 of the first output plane (uniform, or NULL)
  unsigned lo;        // this lane's first column
  const RT* chr0;     // Cb strip rows, this lane's chroma columns
  const RT* chr1;     // Cr
  int j0, r0;
  bool wref;             // store the new reference rows to memory
  RefRows<RT, C>* refv;  // this wave's reference rows (zero for intra frames); the 5/3
                         // colour path leaves the new rows in it
  // n packed words to a plane row; NT: streaming stores (the output is not
  // read again by the decode)
  template <int NWD, bool NT = false>
  __device__ __forceinline__ static void st_words(WV_G RT* p, const uint32_t (&w)[NWD]) {
    if constexpr (NWD == 2) {
      if constexpr (NT) __builtin_nontemporal_store(u32x2{w[0], w[1]}, (WV_G u32x2*)p);
      else *(WV_G u32x2*)p = u32x2{w[0], w[1]};
    } else {
      if constexpr (NT) __builtin_nontemporal_store(w[0], (WV_G uint32_t*)p);
      else *(WV_G uint32_t*)p = w[0];
    }
  }
  // 5/3 YUV420: the reference and RGB words of output rows r, r+1 from their
  // clipped luma y and the strip's chroma bytes.
  template <int J>
  __device__ __forceinline__ void rgb8(const int (&y)[2][C], int r) {
    constexpr int HC = C / 2, NWD = C / 4;
    static_assert(NWD == 1 || NWD == 2, "lane width");
    uint32_t yp[2][HC];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < HC; ++k) yp[h][k] = ypair(y[h][2 * k], y[h][2 * k + 1]);
    if constexpr (WREF) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        uint32_t w[NWD];
#pragma unroll
        for (int m = 0; m < NWD; ++m) {
          w[m] = low_bytes(yp[h][2 * m], yp[h][2 * m + 1]);
          refv->set(2 * J + h, m, w[m]);
        }
        if (wref) st_words<NWD>(at(ref + (r + h) * N, lo), w);
      }
    }
    if (!out) return;
    const int cr_row = (r >> 1) - (r0 >> 1);   // chroma strip row
    uint32_t cbw, crw;
    if constexpr (HC == 4) {
      cbw = *(const uint32_t*)(chr0 + cr_row * (N / 2));
      crw = *(const uint32_t*)(chr1 + cr_row * (N / 2));
    } else {
      cbw = *(const uint16_t*)(chr0 + cr_row * (N / 2));
      crw = *(const uint16_t*)(chr1 + cr_row * (N / 2));
    }
    uint32_t br[HC], bg[HC], bb[HC];
#pragma unroll
    for (int k = 0; k < HC; ++k) {
      const uint32_t cb = (cbw >> (8 * k)) & 0xffu, cr = (crw >> (8 * k)) & 0xffu;
      br[k] = term2(kTermBias + 91881u * 128u - 91881u * cr);
      bg[k] = term2(kTermBias - (22554u + 46802u) * 128u + 22554u * cb + 46802u * cr);
      bb[k] = term2(kTermBias + 116130u * 128u - 116130u * cb);
    }
    constexpr unsigned PL = (unsigned)N * N;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t wr[NWD], wg[NWD], wb[NWD];
#pragma unroll
      for (int m = 0; m < NWD; ++m) {
        const int k0 = 2 * m, k1 = 2 * m + 1;
        wr[m] = low_bytes(clip_add(yp[h][k0], br[k0]), clip_add(yp[h][k1], br[k1]));
        wg[m] = low_bytes(clip_add(yp[h][k0], bg[k0]), clip_add(yp[h][k1], bg[k1]));
        wb[m] = low_bytes(clip_add(yp[h][k0], bb[k0]), clip_add(yp[h][k1], bb[k1]));
      }
      const unsigned o = (unsigned)((r + h) * N);
      st_words<NWD, true>(at(out + o, lo), wr);
      st_words<NWD, true>(at(out + (o + PL), lo), wg);
      st_words<NWD, true>(at(out + (o + 2 * PL), lo), wb);
    }
  }
  template <int J>
  __device__ __forceinline__ void pair(const V (&xe)[C], const V (&xo)[C]) {
    const int r = 2 * (j0 + J);
    V y[2][C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      y[0][c] = clip255(xe[c] + refv->get(2 * J, c));
      y[1][c] = clip255(xo[c] + refv->get(2 * J + 1, c));
    }
    if constexpr (sizeof(RT) == 1 && FMT == WV_YUV420 && C % 4 == 0) {
      rgb8<J>(y, r);
      return;
    }
    if constexpr (WREF) {
      if (wref) {
        st_px<C>(at(ref + r * N, lo), y[0]);
        st_px<C>(at(ref + (r + 1) * N, lo), y[1]);
      }
    }
    if (!out) return;
    if constexpr (FMT == WV_GRAY8) {
      st_px<C>(at(out + r * N, lo), y[0]);
      st_px<C>(at(out + (r + 1) * N, lo), y[1]);
    } else {
      constexpr int HC = C / 2;
      const int cr = (r >> 1) - (r0 >> 1);   // chroma strip row
      V tr[HC], tg[HC], tb[HC];
      V cbv[HC], crv[HC];
      ld_chr<HC>(chr0 + cr * (N / 2), cbv);
      ld_chr<HC>(chr1 + cr * (N / 2), crv);
#pragma unroll
      for (int k = 0; k < HC; ++k) {
        if constexpr (sizeof(RT) == 1) {
          // (Y << 16) + t >> 16 == Y + (t >> 16): the colour terms are per chroma sample
          const int cb = cbv[k] - 128, crr = crv[k] - 128;
          tr[k] = (91881 * crr + 32768) >> 16;
          tg[k] = (-22554 * cb - 46802 * crr + 32768) >> 16;
          tb[k] = (116130 * cb + 32768) >> 16;
        } else {
          const V cb = cbv[k] - 128.0f, crr = crv[k] - 128.0f;
          tr[k] = 1.402f * crr;
          tg[k] = -0.344136f * cb - 0.714136f * crr;
          tb[k] = 1.772f * cb;
        }
      }
      constexpr unsigned PL = (unsigned)N * N;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        V R[C], Gv[C], Bv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          R[c] = clip255(y[h][c] + tr[c >> 1]);
          Gv[c] = clip255(y[h][c] + tg[c >> 1]);
          Bv[c] = clip255(y[h][c] + tb[c >> 1]);
        }
        const unsigned o = (unsigned)((r + h) * N);
        st_px<C>(at(out + o, lo), R);
        st_px<C>(at(out + (o + PL), lo), Gv);
        st_px<C>(at(out + (o + 2 * PL), lo), Bv);
      }
    }
  }
};

// Coefficients of H consecutive samples as loaded (packed int16, or floats).
template <class CT, int H>
struct Packed;
template <>
struct Packed<int16_t, 4> { using T = u32x2; };
template <>
struct Packed<int16_t, 2> { using T = uint32_t; };
template <>
struct Packed<int16_t, 1> { using T = int; };
template <>
struct Packed<float, 4> { using T = f32x4; };
template <>
struct Packed<float, 2> { using T = f32x2; };
template <>
struct Packed<float, 1> { using T = float; };

// Coefficient loads keep the default cache policy: the bands of an
// inter-frame set are read once per frame of the set, and the paper format's
// rebuilt planes are read while still in the memory-side cache, so a
// streaming hint would send those re-reads to HBM.
template <int H>
__device__ __forceinline__ typename Packed<int16_t, H>::T ld_packed(const WV_G int16_t* p) {
  if constexpr (H == 4) return *(const WV_G u32x2*)p;
  else if constexpr (H == 2) return *(const WV_G uint32_t*)p;
  else return (int)*p;
}
template <int H>
__device__ __forceinline__ typename Packed<float, H>::T ld_packed(const WV_G float* p) {
  if constexpr (H == 4) return *(const WV_G f32x4*)p;
  else if constexpr (H == 2) return *(const WV_G f32x2*)p;
  else return *p;
}
// Dequantised values of a packed group (5/3: index * step; 9/7: as stored).
template <int H>
__device__ __forceinline__ void unpack(const typename Packed<int16_t, H>::T& w, int q, int (&v)[H]) {
  if constexpr (H == 4) {
    v[0] = __mul24((int)(int16_t)(w.x & 0xffffu), q);
    v[1] = __mul24((int)w.x >> 16, q);
    v[2] = __mul24((int)(int16_t)(w.y & 0xffffu), q);
    v[3] = __mul24((int)w.y >> 16, q);
  } else if constexpr (H == 2) {
    v[0] = __mul24((int)(int16_t)(w & 0xffffu), q);
    v[1] = __mul24((int)w >> 16, q);
  } else {
    v[0] = __mul24(w, q);
  }
}
template <int H>
__device__ __forceinline__ void unpack(const typename Packed<float, H>::T& w, int, float (&v)[H]) {
  if constexpr (H == 4) {
    v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
  } else if constexpr (H == 2) {
    v[0] = w.x; v[1] = w.y;
  } else {
    v[0] = w;
  }
}

// Inter-frame sets (temporal Haar, Section 3.2): a frame's coefficient is the
// signed sum of three bands at the same position -- the approximation, the
// coarsest detail and the frame's finest detail -- each band a full copy of
// the plane.  5/3: q are signed dequantisation steps, the sum is exact in
// int32; 9/7: q are the signs (+1 / -1, 0 for an absent band).
template <class CT>
struct SetSrc {
  const WV_G CT* b0;
  const WV_G CT* b1;
  const WV_G CT* b2;
  int q0, q1, q2;
};
template <class S>
struct IsSet : std::false_type {};
template <class CT>
struct IsSet<SetSrc<CT>> : std::true_type {};

// H consecutive values already combined at load time.
template <class V, int H>
struct Comb {
  V v[H];
};
template <int H, class V>
__device__ __forceinline__ void unpack(const Comb<V, H>& w, int, V (&v)[H]) {
#pragma unroll
  for (int k = 0; k < H; ++k) v[k] = w.v[k];
}

// The loads of H consecutive coefficients from a source.
template <int H, class CT>
__device__ __forceinline__ typename Packed<CT, H>::T ld_src(const WV_G CT* p, unsigned off) {
  return ld_packed<H>(at(p, off));
}
template <int H>
__device__ __forceinline__ Comb<int, H> ld_src(const SetSrc<int16_t>& s, unsigned off) {
  const auto w0 = ld_packed<H>(at(s.b0, off));
  const auto w1 = ld_packed<H>(at(s.b1, off));
  const auto w2 = ld_packed<H>(at(s.b2, off));
  int v0[H], v1[H], v2[H];
  unpack<H>(w0, s.q0, v0);
  unpack<H>(w1, s.q1, v1);
  unpack<H>(w2, s.q2, v2);
  Comb<int, H> r;
#pragma unroll
  for (int k = 0; k < H; ++k) r.v[k] = v0[k] + v1[k] + v2[k];
  return r;
}
template <int H>
__device__ __forceinline__ Comb<float, H> ld_src(const SetSrc<float>& s, unsigned off) {
  const auto w0 = ld_packed<H>(at(s.b0, off));
  const auto w1 = ld_packed<H>(at(s.b1, off));
  const auto w2 = ld_packed<H>(at(s.b2, off));
  float v0[H], v1[H], v2[H];
  unpack<H>(w0, 0, v0);
  unpack<H>(w1, 0, v1);
  unpack<H>(w2, 0, v2);
  const float s1 = (float)s.q1, s2 = (float)s.q2;
  Comb<float, H> r;
#pragma unroll
  for (int k = 0; k < H; ++k) r.v[k] = (v0[k] + s1 * v1[k]) + s2 * v2[k];
  return r;
}

// The global loads of one segment (see segment below), kept in registers
// so that they can be issued well before the lifting that consumes them.
template <class LF, int N, int K, bool FROM_LL, bool SET = false>
struct SegLoads {
  using CT = typename CoefT<LF>::T;
  static constexpr int H = RL<N>::H, NPUSH = K + LF::D_LO + LF::D_HI;
  using PT = std::conditional_t<SET, Comb<typename LF::V, H>, typename Packed<CT, H>::T>;
  PT s[FROM_LL ? NPUSH : 1], hl[NPUSH], lh[NPUSH], hh[NPUSH];
};

// Band rows of push t (symmetric extension, then a clamp that only matters
// for lane slots past the last segment, whose outputs are discarded).
template <int N>
__device__ __forceinline__ void push_rows(int t, int& rs, int& rd) {
  constexpr int M = N / 2;
  if constexpr (RL<N>::S == 1) {
    // one row per wave (N >= 128): the rows past a segment's last pair lie
    // within a few rows of the level, where one reflection stays in range;
    // no clamp, so the uniform row index stays in scalar registers
    rs = ext_row<N>(2 * t) >> 1;
    rd = ext_row<N>(2 * t + 1) >> 1;
  } else {
    rs = min(max(ext_row<N>(2 * t) >> 1, 0), M - 1);
    rd = min(max(ext_row<N>(2 * t + 1) >> 1, 0), M - 1);
  }
}

// The global loads of one segment: for push i, the low-band row (level L
// only) and the three detail rows, each one vector offset (the lane's column
// plus the row) from the plane's scalar base.
template <class LF, int N, int PP, int K, bool FROM_LL, bool DROP, class SRC, bool SET>
__device__ __forceinline__ void seg_load(const SRC& coef, int g, int j0,
                                         SegLoads<LF, N, K, FROM_LL, SET>& ld) {
  using SL = SegLoads<LF, N, K, FROM_LL, SET>;
  constexpr int H = SL::H, M = N / 2;
  const unsigned lane_s = (unsigned)(g * H), lane_d = (unsigned)(M + g * H);
  static_for<0, SL::NPUSH>([&](auto I) {
    constexpr int i = decltype(I)::value;
    int rs, rd;
    push_rows<N>(j0 - LF::D_LO + i, rs, rd);
    if constexpr (i >= LF::D_LO - LF::S_LO) {
      if constexpr (FROM_LL) ld.s[i] = ld_src<H>(coef, (unsigned)(rs * PP) + lane_s);
      if constexpr (!DROP) ld.hl[i] = ld_src<H>(coef, (unsigned)(rs * PP) + lane_d);
    }
    if constexpr (!DROP) {
      ld.lh[i] = ld_src<H>(coef, (unsigned)((M + rd) * PP) + lane_s);
      ld.hh[i] = ld_src<H>(coef, (unsigned)((M + rd) * PP) + lane_d);
    }
  });
}

// One segment of a level: output pairs [j0, j0 + K) of the level of width N
// (plane edge PP), low-band rows from the LDS window of level l+1 (`s_win`,
// origin row sa) or, at level L, from the stored approximation band; detail
// bands from `ld` (zero when the level is dropped).
template <class LF, int N, int PP, int K, bool FROM_LL, bool DROP, class Emit, bool SET>
__device__ __forceinline__ void seg_run(const SegLoads<LF, N, K, FROM_LL, SET>& ld, int qstep,
                                        const typename LF::V* s_win, int sa, int s_rows, int g,
                                        int j0, Emit& emit) {
  using V = typename LF::V;
  using SL = SegLoads<LF, N, K, FROM_LL, SET>;
  constexpr int H = SL::H, C = RL<N>::C, M = N / 2;
  VStream<LF, C> vs;
  static_for<0, SL::NPUSH>([&](auto I) {
    constexpr int i = decltype(I)::value;
    V top[C], bot[C];
    if constexpr (i >= LF::D_LO - LF::S_LO) {
      V s[H], hl[H];
      if constexpr (FROM_LL) {
        unpack<H>(ld.s[i], qstep, s);
      } else {
        int rs, rd;
        push_rows<N>(j0 - LF::D_LO + i, rs, rd);
        // rows below the window do not occur (it starts at the cone's first
        // row, or at row 0 where the reflection lands); rows past its end
        // feed only pairs that are not emitted
        const int wr = RL<N>::S == 1 ? min(rs - sa, s_rows - 1) : min(max(rs - sa, 0), s_rows - 1);
        ld_lds<H>(s_win + wr * M + g * H, s);
      }
      if constexpr (DROP) {
#pragma unroll
        for (int k = 0; k < H; ++k) hl[k] = V(0);
      } else {
        unpack<H>(ld.hl[i], qstep, hl);
      }
      HLift<LF, N>::run(s, hl, g, top);
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) top[c] = V(0);
    }
    if constexpr (DROP) {
#pragma unroll
      for (int c = 0; c < C; ++c) bot[c] = V(0);
    } else {
      V lh[H], hh[H];
      unpack<H>(ld.lh[i], qstep, lh);
      unpack<H>(ld.hh[i], qstep, hh);
      HLift<LF, N>::run(lh, hh, g, bot);
    }
    vs.template push<i>(top, bot, emit);
  });
}

template <class LF, int N, int PP, int K, bool FROM_LL, bool DROP, class Emit, class SRC>
__device__ __forceinline__ void segment(const SRC& coef, int qstep, const typename LF::V* s_win,
                                        int sa, int s_rows, int g, int j0, Emit& emit) {
  SegLoads<LF, N, K, FROM_LL, IsSet<SRC>::value> ld;
  seg_load<LF, N, PP, K, FROM_LL, DROP>(coef, g, j0, ld);
  seg_run<LF, N, PP, K, FROM_LL, DROP>(ld, qstep, s_win, sa, s_rows, g, j0, emit);
}

// Output pairs of level l in the cone of a strip of `rows` rows whose start
// is aligned: the rows level l-1 reads from it, rounded up to even.
template <class LF>
constexpr int cone_pairs(int rows, int l) {
  int w = rows;
  for (int k = 1; k < l; ++k) {
    const int n = w / 2 + LF::S_LO + LF::S_HI;
    w = n + (n & 1);
  }
  return w / 2;
}

// Pairs per segment of level l (width N) of a plane whose strips have `rows`
// rows, dealt to `nw` waves.  A segment of K pairs takes K + D_LO + D_HI
// pushes, so the pushes per pair fall as K grows; K is the smallest that
// covers the cone's pairs in one round of tasks: one pair per task where
// several rows sit side by side in a wave (their tasks fill the row slots),
// else the pairs split evenly over the waves (at most 4 per segment).
template <class LF, int N, int ROWS, int l, int NWV>
constexpr int seg_pairs() {
  constexpr int np = cone_pairs<LF>(ROWS, l), slots = RL<N>::S * NWV;
  if constexpr (RL<N>::S > 1) {
    constexpr int k = (np + slots - 1) / slots;
    return k < 1 ? 1 : k;
  } else {
    constexpr int k = (np + NWV - 1) / NWV;
    return k > 4 ? 4 : (k < 1 ? 1 : k);
  }
}

// Level l of one plane: the pairs of its cone rows [a, b) in segments of K,
// dealt to `nwp` waves (this wave is number `rank` among them; with several
// rows per wave each lane slot takes its own segment).
// The loads of level l of a plane (one row per wave) for this wave's first
// segment: issued early by the caller, consumed by `level` (argument pre).
template <class LF, int PP, int L, int l, int K, class SRC>
using PreLoads = SegLoads<LF, (PP >> (l - 1)), K, l == L, IsSet<SRC>::value>;

template <class LF, int PP, int L, int l, int K, class SRC>
__device__ __forceinline__ void level_preload(const Plane<LF, L, SRC>& pl, int lc, int rank, int lane,
                                              PreLoads<LF, PP, L, l, K, SRC>& ld) {
  constexpr int N = PP >> (l - 1);
  static_assert(RL<N>::S == 1, "one row per wave");
  const int j0 = (pl.a[l] >> 1) + rank * K;
  if (l <= L - lc)
    seg_load<LF, N, PP, K, l == L, true>(pl.coef, lane, j0, ld);
  else
    seg_load<LF, N, PP, K, l == L, false>(pl.coef, lane, j0, ld);
}

template <class LF, int PP, int L, int l, int K, class MakeEmit, class SRC, class Pre = std::nullptr_t>
__device__ __forceinline__ void level(const Plane<LF, L, SRC>& pl, int qstep, int lc, int rank,
                                      int nwp, int lane, MakeEmit&& make_emit, const Pre* pre = nullptr) {
  constexpr int N = PP >> (l - 1);
  using RLN = RL<N>;
  constexpr int S = RLN::S, G = RLN::G;
  // one row per wave: the row slot is 0 and every row index stays scalar
  const int g = S == 1 ? lane : lane % G, q = S == 1 ? 0 : lane / G;
  const int np = (pl.b[l] - pl.a[l]) >> 1;
  const int ntask = (np + K - 1) / K;
  const bool drop = l <= L - lc;
  const typename LF::V* s_win = nullptr;
  int sa = 0, srows = 1;
  if constexpr (l < L) {
    s_win = pl.win[(l + 1) & 1];
    sa = pl.a[l + 1];
    srows = pl.b[l + 1] - pl.a[l + 1];
  }
  for (int t0 = rank * S; t0 < ntask; t0 += nwp * S) {
    const int t = t0 + q;
    const int j0 = (pl.a[l] >> 1) + t * K;
    auto emit = make_emit(g, j0, min(max(np - t * K, 0), K));
    if constexpr (!std::is_same<Pre, std::nullptr_t>::value) {
      if (t0 == rank * S) {   // this wave's first segment: its loads are in *pre
        if (drop)
          seg_run<LF, N, PP, K, l == L, true>(*pre, qstep, s_win, sa, srows, g, j0, emit);
        else
          seg_run<LF, N, PP, K, l == L, false>(*pre, qstep, s_win, sa, srows, g, j0, emit);
        continue;
      }
    }
    if (drop)
      segment<LF, N, PP, K, l == L, true>(pl.coef, qstep, s_win, sa, srows, g, j0, emit);
    else
      segment<LF, N, PP, K, l == L, false>(pl.coef, qstep, s_win, sa, srows, g, j0, emit);
  }
}

template <class LF, int PP, int L, int l, int K, class SRC, class Pre = std::nullptr_t>
__device__ __forceinline__ void coarse_level(const Plane<LF, L, SRC>& pl, int qstep, int lc,
                                             int rank, int nwp, int lane, const Pre* pre = nullptr) {
  constexpr int N = PP >> (l - 1), C = RL<N>::C;
  using V = typename LF::V;
  V* win = pl.win[l & 1];
  const int a = pl.a[l];
  level<LF, PP, L, l, K>(pl, qstep, lc, rank, nwp, lane, [&](int g, int j0, int kk) {
    return ToWindow<V, N, C>{win + g * C, j0, kk, a};
  }, pre);
}

// Reference rows of a segment's pairs, fetched before the lifting starts.
template <int K, class RT, class RR>
__device__ __forceinline__ void prefetch_ref(const WV_G RT* ref, unsigned lo, int N, int j0, RR& refv) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    refv.load(2 * j, at(ref + 2 * (j0 + j) * N, lo));
    refv.load(2 * j + 1, at(ref + (2 * (j0 + j) + 1) * N, lo));
  }
}

// Reference rows of a segment's pairs from the strip's chroma rows in LDS,
// which hold the previous frame's reconstruction (GOP form).
template <int K, class RT, class RR>
__device__ __forceinline__ void prefetch_chr(const RT* chr, int N, int j0, int r0, RR& refv) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    refv.load_lds(2 * j, chr + (2 * (j0 + j) - r0) * N);
    refv.load_lds(2 * j + 1, chr + (2 * (j0 + j) + 1 - r0) * N);
  }
}

// Barrier for LDS hand-over between phases.  The fences are restricted to
// LDS, so the barrier does not wait for outstanding global memory operations
// (stores of reference and output rows, loads the compiler issued early).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Ordering of one wave's LDS writes before its own later reads (DS
// instructions of a wave execute in order; this only keeps the compiler from
// moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// SCHED 0: phase k computes luma level L+1-k and chroma level L-k on all
// waves, one barrier per phase.  SCHED 1: each plane's coarse levels run as a
// chain on one wave (luma L..3 on wave 0, chroma L..2 on waves 1 and 2) with
// no barrier between levels; then luma level 2 with the finest chroma rows;
// then the finest luma rows: three phases.
// Coefficient source of plane p of a job's tile: the stored plane, or (SET)
// the three bands of an inter-frame set that make up the job's frame.
template <class CT, bool SET>
__device__ __forceinline__ std::conditional_t<SET, SetSrc<CT>, const WV_G CT*> plane_src(
    const Job& job, int p, size_t tile_off, size_t band_elems) {
  const WV_G CT* b = uniform((const WV_G CT*)job.coef[p] + tile_off);
  if constexpr (SET)
    return SetSrc<CT>{b, b + band_elems, b + (size_t)job.hband * band_elems, job.qstep, job.hq[0],
                      job.hq[1]};
  else
    return b;
}

// first / last: the unit's first and last frame in this launch.  In the GOP
// form a strip's reference rows stay on chip between its frames (luma in the
// waves' registers `lkeep` for 8-bit samples, chroma in the strip's LDS rows)
// and reach memory only after the last frame.
template <class LF, int FMT, int P, int L, int R, int NW, int SCHED, bool SET>
__device__ __forceinline__ void strip_unit(Smem<LF, FMT, P, L, R, SCHED>& sm, const WorkArgs& a, int unit,
                                           int frame, bool first, bool last,
                                           RefRows<typename CoefT<LF>::R, RL<P>::C>& lkeep) {
  using V = typename LF::V;
  using CT = typename CoefT<LF>::T;
  using RT = typename CoefT<LF>::R;
  constexpr int NST = P / R;
  constexpr bool YUV = FMT == WV_YUV420;
  constexpr int PC = P / 2, RC = R / 2;
  static_assert(!YUV || NW >= 3, "luma and both chroma planes need a wave each");
  const int it = unit / NST, st = unit - it * NST;
  const Item item = a.items_dev ? a.items_dev[it] : a.items[it];
  const int jf = frame < 0 ? item.job : frame;
  const Job& job = a.jobs_dev ? a.jobs_dev[jf] : a.jobs[jf];
  const int lc = item.lc, qs = job.qstep;
  // inter-frame-set frames stand alone: no reference is read or written
  const bool intra = SET || (job.flags & kJobIntra) != 0;
  const bool has_out = (job.flags & kJobHasOut) != 0;
  constexpr bool KEEPY = sizeof(RT) == 1 && YUV && !SET, KEEPC = YUV && !SET;
  const bool wref_y = !KEEPY || last, wref_c = !KEEPC || last;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));

  using SrcT = std::conditional_t<SET, SetSrc<CT>, const WV_G CT*>;
  Plane<LF, L, SrcT> py;
  py.coef = plane_src<CT, SET>(job, 0, (size_t)item.tile * P * P, job.hstride);
  py.ref = uniform((WV_G RT*)job.ref[0] + (size_t)item.tile * P * P);
  py.win[0] = sm.ya();
  py.win[1] = sm.yb;
  cone<LF, L>(st * R, R, P, py.a, py.b);
  Plane<LF, L, SrcT> pc[2];
  if constexpr (YUV) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      pc[p].coef = plane_src<CT, SET>(job, 1 + p, (size_t)item.tile * PC * PC, job.hstride / 4);
      pc[p].ref = uniform((WV_G RT*)job.ref[1 + p] + (size_t)item.tile * PC * PC);
      pc[p].win[0] = sm.ca[p];
      pc[p].win[1] = sm.cb(p);
      cone<LF, L>(st * RC, RC, PC, pc[p].a, pc[p].b);
    }
  }

  // The finest luma level: one segment of K1 pairs per wave.
  constexpr int K1 = R / 2 / NW, C1 = RL<P>::C;
  static_assert(K1 >= 1 && K1 <= 8 && (R / 2) % NW == 0, "strip rows per wave");
  static_assert(RL<P>::G == 64, "one luma row per wave");
  const int j0y = (py.a[1] >> 1) + wave * K1;
  const bool drop1 = 1 <= L - lc;
  SegLoads<LF, P, K1, L == 1, SET> ly;
  LumaOut<LF, FMT, P, C1, !SET> lout;
  {
    WV_G RT* outp = has_out ? (WV_G RT*)job.out + (size_t)item.slot * (YUV ? 3 : 1) * P * P : nullptr;
    lout.ref = py.ref;
    lout.out = outp ? uniform(outp) : nullptr;
    lout.lo = (unsigned)(lane * C1);
    lout.chr0 = sm.chr[0] + lane * (C1 / 2);
    lout.chr1 = sm.chr[YUV ? 1 : 0] + lane * (C1 / 2);
    lout.j0 = j0y;
    lout.r0 = st * R;
    lout.wref = wref_y;
    lout.refv = &lkeep;
  }

  if constexpr (SCHED == 1) {
    // the finest luma rows of this wave (the last phase of every schedule)
    // 5/3 stored frames: its loads go out at the start of the frame and
    // arrive while the coarse levels are computed (the 9/7 and set forms hold
    // their loads unpacked, too many registers to carry through the chains)
    constexpr bool EARLY = std::is_same<LF, Inv53>::value && !SET;
    auto luma1_load = [&]() __attribute__((always_inline)) {
      if (drop1)
        seg_load<LF, P, P, K1, L == 1, true>(py.coef, lane, j0y, ly);
      else
        seg_load<LF, P, P, K1, L == 1, false>(py.coef, lane, j0y, ly);
    };
    auto luma1 = [&]() __attribute__((always_inline)) {
      if constexpr (!EARLY) luma1_load();
      if (intra) lkeep.template zero<K1>();
      else if (!KEEPY || first) prefetch_ref<K1>(lout.ref, lout.lo, P, j0y, lkeep);
      const typename LF::V* sw = nullptr;
      int sa = 0, srows = 1;
      if constexpr (L > 1) {
        sw = py.win[0];
        sa = py.a[2];
        srows = py.b[2] - py.a[2];
      }
      if (drop1)
        seg_run<LF, P, P, K1, L == 1, true>(ly, qs, sw, sa, srows, lane, j0y, lout);
      else
        seg_run<LF, P, P, K1, L == 1, false>(ly, qs, sw, sa, srows, lane, j0y, lout);
    };
    // the finest rows of chroma plane pi
    auto chroma1 = [&](auto PI, int rank, int nwp) __attribute__((always_inline)) {
      constexpr int pi = decltype(PI)::value;
      constexpr int KC = 4, C = RL<PC>::C;
      const Plane<LF, L, SrcT>& pl = pc[pi];
      RT* chr = sm.chr[pi];
      level<LF, PC, L, 1, KC>(pl, qs, lc, rank, nwp, lane, [&](int g, int j0, int) {
        ChromaOut<LF, PC, C, !SET> e;
        e.ref = pl.ref;
        e.lo = (unsigned)(g * C);
        e.chr = chr + g * C;
        e.j0 = j0;
        e.r0 = st * RC;
        e.wref = wref_c;
        if (intra) e.refv.template zero<KC>();
        else if (!KEEPC || first) prefetch_ref<KC>(e.ref, e.lo, PC, j0, e.refv);
        else prefetch_chr<KC>(e.chr, PC, j0, e.r0, e.refv);
        return e;
      });
    };

    // Wave priority falls with the distance to the output (3 for the coarse
    // chains, 1 for the middle phase, 0 for the finest rows).  The chains are
    // short dependent runs on a few waves while the other workgroups of the
    // CU stream their finest rows: issued first, they bring their workgroup to
    // its next barrier sooner, and the finest rows take the slots left over.
    // A: coarse chains, one wave per plane
    constexpr bool phase_a = L >= 3 || (YUV && L >= 2);
    if constexpr (EARLY) luma1_load();
    __builtin_amdgcn_s_setprio(3);
    if constexpr (L >= 3) {
      if (wave == 0) {
        static_for_down<L, 2>([&](auto LL) {
          constexpr int l = decltype(LL)::value;
          coarse_level<LF, P, L, l, seg_pairs<LF, (P >> (l - 1)), R, l, 1>()>(py, qs, lc, 0, 1, lane);
          wave_lds_sync();
        });
      }
    }
    if constexpr (YUV && L >= 2) {
      static_for<0, 2>([&](auto PI) {
        constexpr int pi = decltype(PI)::value;
        if (wave == 1 + pi) {
          static_for_down<L, 1>([&](auto LL) {
            constexpr int l = decltype(LL)::value;
            coarse_level<LF, PC, L, l, seg_pairs<LF, (PC >> (l - 1)), RC, l, 1>()>(pc[pi], qs, lc, 0, 1, lane);
            wave_lds_sync();
          });
        }
      });
    }
    if constexpr (phase_a) lds_barrier();
    __builtin_amdgcn_s_setprio(1);
    // B: luma level 2 on the waves not busy with chroma, the finest chroma
    // rows on waves 1 and 2
    if constexpr (L >= 2 || YUV) {
      const bool cwave = YUV && (wave == 1 || wave == 2);
      if constexpr (L >= 2) {
        if (!cwave) {
          const int rank = YUV ? (wave == 0 ? 0 : wave - 2) : wave, nwp = YUV ? NW - 2 : NW;
          coarse_level<LF, P, L, 2, seg_pairs<LF, (P >> 1), R, 2, YUV ? NW - 2 : NW>()>(py, qs, lc, rank, nwp, lane);
        }
      }
      if constexpr (YUV) {
        static_for<0, 2>([&](auto PI) {
          if (wave == 1 + decltype(PI)::value) chroma1(PI, 0, 1);
        });
      }
      lds_barrier();
    }
    // C: the finest luma rows
    __builtin_amdgcn_s_setprio(0);
    luma1();
    return;
  }

  // Phase k: luma level L+1-k and chroma level L-k.
  static_for<0, L + 1>([&](auto KK) {
    constexpr int k = decltype(KK)::value;
    constexpr int ly_l = L + 1 - k, lcv = L - k;
    constexpr bool do_y = ly_l >= 1 && ly_l <= L, do_c = YUV && lcv >= 1;
    // wave priority by distance to the output, as in the chain schedule
    __builtin_amdgcn_s_setprio(ly_l >= 3 ? 3 : ly_l == 2 ? 1 : 0);
    if constexpr (do_y || do_c) {
      // waves per plane: luma alone, chroma alone (two planes) or all three
      int plane = 0, rank = wave, nwp = NW;
      if constexpr (do_y && do_c) {
        plane = wave % 3;
        rank = wave / 3;
        nwp = (NW - plane + 2) / 3;
      } else if constexpr (do_c) {
        plane = 1 + (wave & 1);
        rank = wave >> 1;
        nwp = (NW - (wave & 1) + 1) / 2;
      }
      if constexpr (do_y) {
        if (plane == 0) {
          if constexpr (ly_l >= 2) {
            coarse_level<LF, P, L, ly_l, seg_pairs<LF, (P >> (ly_l - 1)), R, ly_l, (do_c ? (NW + 2) / 3 : NW)>()>(py, qs, lc, rank, nwp, lane);
          } else {
            if (drop1)
              seg_load<LF, P, P, K1, L == 1, true>(py.coef, lane, j0y, ly);
            else
              seg_load<LF, P, P, K1, L == 1, false>(py.coef, lane, j0y, ly);
            if (intra) lkeep.template zero<K1>();
            else if (!KEEPY || first) prefetch_ref<K1>(lout.ref, lout.lo, P, j0y, lkeep);
            const typename LF::V* sw = nullptr;
            int sa = 0, srows = 1;
            if constexpr (L > 1) {
              sw = py.win[0];
              sa = py.a[2];
              srows = py.b[2] - py.a[2];
            }
            if (drop1)
              seg_run<LF, P, P, K1, L == 1, true>(ly, qs, sw, sa, srows, lane, j0y, lout);
            else
              seg_run<LF, P, P, K1, L == 1, false>(ly, qs, sw, sa, srows, lane, j0y, lout);
          }
        }
      }
      if constexpr (do_c) {
        // one instance per chroma plane: the plane's state stays in registers
        static_for<0, 2>([&](auto PI) {
          constexpr int pi = decltype(PI)::value;
          if (plane == 1 + pi) {
            const Plane<LF, L, SrcT>& pl = pc[pi];
            if constexpr (lcv >= 2) {
              coarse_level<LF, PC, L, lcv, seg_pairs<LF, (PC >> (lcv - 1)), RC, lcv, (do_y ? (NW + 2) / 3 : (NW + 1) / 2)>()>(pl, qs, lc, rank, nwp, lane);
            } else {
              constexpr int KC = 4, C = RL<PC>::C;
              RT* chr = sm.chr[pi];
              level<LF, PC, L, 1, KC>(pl, qs, lc, rank, nwp, lane, [&](int g, int j0, int) {
                ChromaOut<LF, PC, C, !SET> e;
                e.ref = pl.ref;
                e.lo = (unsigned)(g * C);
                e.chr = chr + g * C;
                e.j0 = j0;
                e.r0 = st * RC;
                e.wref = wref_c;
                if (intra) e.refv.template zero<KC>();
                else if (!KEEPC || first) prefetch_ref<KC>(e.ref, e.lo, PC, j0, e.refv);
                else prefetch_chr<KC>(e.chr, PC, j0, e.r0, e.refv);
                return e;
              });
            }
          }
        });
      }
      if constexpr (k < L) lds_barrier();
    }
  });
}


// WPE: waves per SIMD the register allocation must leave room for.
// One work unit: a tile strip of one frame, or (GOP form, a.n_frames > 0)
// the same tile strip through consecutive frames.  A strip's reference rows
// are written and read again by the same waves, and the barrier between
// frames orders them: frames of one strip need no other synchronisation, so
// workgroups drift apart in phase and overlap each other's latencies.
template <class LF, int FMT, int P, int L, int R, int NW, int SCHED, bool SET>
__device__ __forceinline__ void strip_work(Smem<LF, FMT, P, L, R, SCHED>& sm, const WorkArgs& a,
                                           int unit) {
  const int nf = a.n_frames > 0 ? a.n_frames : 1;
  RefRows<typename CoefT<LF>::R, RL<P>::C> lkeep;   // this wave's luma reference rows
  for (int f = 0; f < nf; ++f) {
    if (f) __syncthreads();
    // An opaque copy of the unit index: the unit's geometry (item, cones,
    // plane pointers) is recomputed per frame instead of being held live in
    // registers across the whole frame loop.
    // (unit is uniform: every lane of the workgroup holds the same value).
    int u = __builtin_amdgcn_readfirstlane(unit);
    asm volatile("" : "+s"(u));
    strip_unit<LF, FMT, P, L, R, NW, SCHED, SET>(sm, a, u, a.n_frames > 0 ? f : -1, f == 0, f == nf - 1,
                                                 lkeep);
  }
}

template <class LF, int FMT, int P, int L, int R, int NW, bool PERSIST, int WPE, int SCHED,
          bool SET>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_strip(const WorkArgs a) {
  __shared__ Smem<LF, FMT, P, L, R, SCHED> sm;
  const int total = a.total_dev ? *a.total_dev : a.total;
  if (!PERSIST) {
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    if (u < total) strip_work<LF, FMT, P, L, R, NW, SCHED, SET>(sm, a, u);
    return;
  }
  __shared__ int s_unit;
  for (;;) {
    if (threadIdx.x == 0) s_unit = (int)atomicAdd(&a.counter[0], 1u);
    __syncthreads();
    const int u = s_unit;
    __syncthreads();
    if (u >= total) break;
    strip_work<LF, FMT, P, L, R, NW, SCHED, SET>(sm, a, u);
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

}  // namespace strip
}  // namespace wv
