// Device-side lifting building blocks shared by the fused, plain and encoder
// kernels: symmetric extension and one output pair of each 1D transform.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wv {

// Whole-sample symmetric extension of a length-n signal (n >= 2):
// x[-j] = x[j], x[n-1+j] = x[n-1-j].  Returns the source index in [0, n).
__device__ __forceinline__ int wss(int j, int n) {
  const int p = 2 * n - 2;
  if (p <= 0) return 0;
  while (j < 0 || j >= n) {
    if (j < 0) j = -j;
    if (j >= n) j = p - j;
  }
  return j;
}
// Index into the low band (even samples) / high band (odd samples) of a
// length-n signal, for an extended band index i.
__device__ __forceinline__ int s_idx(int i, int n) { return wss(2 * i, n) >> 1; }
__device__ __forceinline__ int d_idx(int i, int n) { return wss(2 * i + 1, n) >> 1; }

// --------------------------------------------------------------- inverse 5/3
// One output pair x[2k], x[2k+1] from s[k..k+1] and d[k-1..k+1]
// (JPEG 2000 reversible lifting: undo the update, then the predict).
struct Inv53 {
  using V = int;
  static constexpr int S_LO = 0, S_HI = 1, D_LO = 1, D_HI = 1;
  static constexpr int NS = 2, ND = 3;
  __device__ static __forceinline__ void pair(const V* s, const V* d, V& xe, V& xo) {
    const int e0 = s[0] - ((d[0] + d[1] + 2) >> 2);
    const int e1 = s[1] - ((d[1] + d[2] + 2) >> 2);
    xe = e0;
    xo = d[1] + ((e0 + e1) >> 1);
  }
  // NP consecutive output pairs x[0 .. 2NP) from s[0 .. NP] and d[0 .. NP+1]
  // (s[i] = s_{k+i}, d[i] = d_{k-1+i} for the first pair k).
  template <int NP>
  __device__ static __forceinline__ void run(const V* s, const V* d, V* x) {
    V e[NP + 1];
#pragma unroll
    for (int i = 0; i <= NP; ++i) e[i] = s[i] - ((d[i] + d[i + 1] + 2) >> 2);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      x[2 * i] = e[i];
      x[2 * i + 1] = d[i + 1] + ((e[i] + e[i + 1]) >> 1);
    }
  }
};

// --------------------------------------------------------------- inverse 9/7
// CDF 9/7 irreversible lifting constants (JPEG 2000 Part 1).
#define WV_A97 (-1.586134342059924)
#define WV_B97 (-0.052980118572961)
#define WV_G97 (0.882911075530934)
#define WV_D97 (0.443506852043971)
#define WV_K97 (1.230174104914001)

// One output pair x[2k], x[2k+1] from s[k-1..k+2] and d[k-2..k+2]:
// scale (low by K, high by 1/K), then undo delta, gamma, beta, alpha.
struct Inv97 {
  using V = float;
  static constexpr int S_LO = 1, S_HI = 2, D_LO = 2, D_HI = 2;
  static constexpr int NS = 4, ND = 5;
  __device__ static __forceinline__ void pair(const V* s, const V* d, V& xe, V& xo) {
    const float K = (float)WV_K97, IK = (float)(1.0 / WV_K97);
    const float A = (float)WV_A97, B = (float)WV_B97, G = (float)WV_G97, D = (float)WV_D97;
    const float om2 = d[0] * IK, om1 = d[1] * IK, o0 = d[2] * IK, o1 = d[3] * IK, o2 = d[4] * IK;
    const float em1 = K * s[0] - D * (om2 + om1);
    const float e0 = K * s[1] - D * (om1 + o0);
    const float e1 = K * s[2] - D * (o0 + o1);
    const float e2 = K * s[3] - D * (o1 + o2);
    const float pm1 = om1 - G * (em1 + e0);
    const float p0 = o0 - G * (e0 + e1);
    const float p1 = o1 - G * (e1 + e2);
    const float f0 = e0 - B * (pm1 + p0);
    const float f1 = e1 - B * (p0 + p1);
    xe = f0;
    xo = p0 - A * (f0 + f1);
  }
  // NP consecutive output pairs from s[0 .. NP+2] (s_{k-1+i}) and
  // d[0 .. NP+3] (d_{k-2+i}); intermediate index t of the paper's-order
  // lifting steps is stored at t + offset.
  template <int NP>
  __device__ static __forceinline__ void run(const V* s, const V* d, V* x) {
    const float K = (float)WV_K97, IK = (float)(1.0 / WV_K97);
    const float A = (float)WV_A97, B = (float)WV_B97, G = (float)WV_G97, D = (float)WV_D97;
    float o0[NP + 4], e1[NP + 3], o1[NP + 2], e2[NP + 1];
#pragma unroll
    for (int t = 0; t < NP + 4; ++t) o0[t] = d[t] * IK;           // t-2
#pragma unroll
    for (int t = 0; t < NP + 3; ++t) e1[t] = K * s[t] - D * (o0[t] + o0[t + 1]);   // t-1
#pragma unroll
    for (int t = 0; t < NP + 2; ++t) o1[t] = o0[t + 1] - G * (e1[t] + e1[t + 1]); // t-1
#pragma unroll
    for (int t = 0; t < NP + 1; ++t) e2[t] = e1[t + 1] - B * (o1[t] + o1[t + 1]); // t
#pragma unroll
    for (int t = 0; t < NP; ++t) {
      x[2 * t] = e2[t];
      x[2 * t + 1] = o1[t + 1] - A * (e2[t] + e2[t + 1]);
    }
  }
};

// --------------------------------------------------------------- forward 5/3
// Low/high output k of a line read through x(i) (any index; the accessor
// applies the symmetric extension).
struct Fwd53 {
  using V = int;
  template <class X>
  __device__ static __forceinline__ void pair(X x, int k, V& s, V& d) {
    const int xm2 = x(2 * k - 2), xm1 = x(2 * k - 1), x0 = x(2 * k), x1 = x(2 * k + 1),
              x2 = x(2 * k + 2);
    const int dk = x1 - ((x0 + x2) >> 1);
    const int dkm1 = xm1 - ((xm2 + x0) >> 1);
    d = dk;
    s = x0 + ((dkm1 + dk + 2) >> 2);
  }
};

// --------------------------------------------------------------- forward 9/7
struct Fwd97 {
  using V = double;
  template <class X>
  __device__ static __forceinline__ void pair(X x, int k, V& s, V& d) {
    const double A = WV_A97, B = WV_B97, G = WV_G97, D = WV_D97, K = WV_K97;
    const double em2 = x(2 * k - 4), em1 = x(2 * k - 2), e0 = x(2 * k), e1 = x(2 * k + 2),
                 e2 = x(2 * k + 4);
    const double om2 = x(2 * k - 3), om1 = x(2 * k - 1), o0 = x(2 * k + 1), o1 = x(2 * k + 3);
    const double p_m2 = om2 + A * (em2 + em1);
    const double p_m1 = om1 + A * (em1 + e0);
    const double p_0 = o0 + A * (e0 + e1);
    const double p_1 = o1 + A * (e1 + e2);
    const double f_m1 = em1 + B * (p_m2 + p_m1);
    const double f_0 = e0 + B * (p_m1 + p_0);
    const double f_1 = e1 + B * (p_0 + p_1);
    const double q_m1 = p_m1 + G * (f_m1 + f_0);
    const double q_0 = p_0 + G * (f_0 + f_1);
    const double g_0 = f_0 + D * (q_m1 + q_0);
    s = g_0 / K;
    d = q_0 * K;
  }
};

}  // namespace wv
