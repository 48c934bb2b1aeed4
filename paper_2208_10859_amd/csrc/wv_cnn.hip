// Restoration network on decoded viewports: four 3x3 convolutions (3 -> 32
// -> 32 -> 32 -> 3), ReLU after the first three, residual skip.  Forward,
// backward and the optimiser step are hand-written kernels; the convolutions
// are implicit GEMMs on bfloat16 MFMA (v_mfma_f32_16x16x32_bf16) with fp32
// accumulation.  Images and activations are NHWC; three-channel images are
// stored with a fourth zero channel so that a pixel is 8 bytes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "wv_cnn.h"
#include "wv_ctx.h"

namespace wv {
namespace cnn {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int HID = 32;
constexpr int BH = 8, BW = 32;            // weight gradients: pixels per block, 8 rows x 32 columns

// float -> bfloat16, round to nearest, ties to even (finite values)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int kpad16(int cin) { return (9 * cin + 15) / 16 * 16; }

// The backward data pass of one layer (the convolution of the output
// gradient with the flipped, transposed kernel, masked by the layer's ReLU)
// as an implicit GEMM on gfx950's
// v_mfma_f32_16x16x32_bf16: M = output channels (16 per MFMA), N = pixels
// (16 consecutive columns of one row), K = 9 taps x input channels,
// tap-major, padded to a multiple of 32.  For 32 input channels one K step is
// one tap; for 4 it is 8 taps.  MFMA 16x16x32 operands: lane l supplies
// A[l % 16][8 (l / 16) + q] and B[8 (l / 16) + q][l % 16], q = 0..7 (any
// pairing of K positions works as long as A and B use the same one), and
// receives D[4 (l / 16) + q][l % 16]: four consecutive output channels of
// one pixel, stored as one 8-byte write.
// A workgroup computes a 16 x 32 pixel block; wave w owns rows 4w .. 4w+3
// (eight 16-pixel blocks).  Each wave holds the layer's whole weight matrix
// in registers (18 operands of 8 bf16 for 32 -> 32), loaded once; the input
// patch with its one-pixel border is staged in LDS, for 32 channels as four
// planes of 8-channel (16-byte) pixels so that the 16 lanes of an operand
// read 16 consecutive 16-byte words.
//   out = bf16(aux > 0 ? acc : 0)   [pixels][COUT]   (aux: the layer's input activation)
constexpr int CH = 16, CW = 32;           // output pixels per workgroup: 16 rows x 32 columns
constexpr int kpad32(int cin) { return (9 * cin + 31) / 32 * 32; }

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf8 as_bf8(uint4 v) { return __builtin_bit_cast(bf8, v); }

// Two floats to a packed bfloat16 pair, rounded to nearest even (one
// v_cvt_pk_bf16_f32; the same result as f2bf for finite values).
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf2));
}

template <int CIN, int COUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv(const uint16_t* __restrict__ x,
                                              const uint16_t* __restrict__ wt,
                                              const uint16_t* __restrict__ aux, uint16_t* __restrict__ out,
                                              int N, int H, int W) {
  static_assert(CIN == 4 || CIN == 32, "input channels: 4 or 32");
  constexpr int KP = kpad32(CIN), KS = KP / 32, NB = COUT / 16;
  constexpr int PW = CW + 2, PH = CH + 2, PLANE = PH * PW + 1;
  constexpr int LDS_BYTES = CIN == 32 ? 4 * PLANE * 16 : PH * PW * 8;
  __shared__ __align__(16) unsigned char lds[LDS_BYTES];
  const int nbx = (W + CW - 1) / CW, nby = (H + CH - 1) / CH;
  const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, n = blockIdx.x / (nbx * nby);
  const int y0 = by * CH, x0 = bx * CW;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, i16 = lane & 15, g = lane >> 4;

  // the weight matrix, in registers for the whole block
  bf8 wr[KS][NB];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      wr[ks][nb] = as_bf8(*(const uint4*)(wt + (nb * 16 + i16) * KP + ks * 32 + 8 * g));

  // input patch with a one-pixel border (zero outside the image); every
  // global read is issued before the LDS writes, so that the staging waits
  // for memory once
  if constexpr (CIN == 32) {
    constexpr int NI = PH * PW * 4, NIT = (NI + 255) / 256;
    uint4 pv[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = tid + 256 * it, p = idx >> 2, c = idx & 3;
      const int pr = p / PW, pc = p - pr * PW;
      const int gy = y0 + pr - 1, gx = x0 + pc - 1;
      pv[it] = make_uint4(0u, 0u, 0u, 0u);
      if (idx < NI && gy >= 0 && gy < H && gx >= 0 && gx < W)
        pv[it] = *(const uint4*)(x + ((size_t)(n * H + gy) * W + gx) * 32 + c * 8);
    }
    uint4* p16 = (uint4*)lds;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = tid + 256 * it;
      if (idx < NI) p16[(idx & 3) * PLANE + (idx >> 2)] = pv[it];
    }
  } else {
    constexpr int NI = PH * PW, NIT = (NI + 255) / 256;
    uint2 pv[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int p = tid + 256 * it, pr = p / PW, pc = p - pr * PW;
      const int gy = y0 + pr - 1, gx = x0 + pc - 1;
      pv[it] = make_uint2(0u, 0u);
      if (p < NI && gy >= 0 && gy < H && gx >= 0 && gx < W)
        pv[it] = *(const uint2*)(x + ((size_t)(n * H + gy) * W + gx) * 4);
    }
    uint2* p8 = (uint2*)lds;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int p = tid + 256 * it;
      if (p < NI) p8[p] = pv[it];
    }
  }
  __syncthreads();

  f4 acc[8][NB];
#pragma unroll
  for (int mb = 0; mb < 8; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
    for (int mb = 0; mb < 8; ++mb) {
      const int r = 4 * wave + (mb >> 1), c = (mb & 1) * 16 + i16;
      uint4 bv;
      if constexpr (CIN == 32) {
        const int ky = ks / 3, kx = ks - 3 * (ks / 3);
        bv = ((const uint4*)lds)[g * PLANE + (r + ky) * PW + c + kx];
      } else {
        // taps t0 = 8 ks + 2 g and t0 + 1, four channels each; taps >= 9 are zero
        const uint2* p8 = (const uint2*)lds;
        const int t0 = ks * 8 + 2 * g, t1 = t0 + 1;
        const int u0 = min(t0, 8), u1 = min(t1, 8);
        uint2 lo = p8[(r + u0 / 3) * PW + c + u0 % 3];
        uint2 hi = p8[(r + u1 / 3) * PW + c + u1 % 3];
        if (t0 >= 9) lo = make_uint2(0u, 0u);
        if (t1 >= 9) hi = make_uint2(0u, 0u);
        bv = make_uint4(lo.x, lo.y, hi.x, hi.y);
      }
      const bf8 b = as_bf8(bv);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[ks][nb], b, acc[mb][nb], 0, 0, 0);
    }
  }

  // epilogue: lane (g, i16) holds channels nb * 16 + 4 g .. + 3 of pixel i16
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    const int gy = y0 + 4 * wave + (mb >> 1), gx = x0 + (mb & 1) * 16 + i16;
    if (gy >= H || gx >= W) continue;
    const size_t px = (size_t)(n * H + gy) * W + gx;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const size_t o = px * COUT + nb * 16 + 4 * g;
      const uint2 m = *(const uint2*)(aux + o);
      const uint16_t mh[4] = {(uint16_t)m.x, (uint16_t)(m.x >> 16), (uint16_t)m.y, (uint16_t)(m.y >> 16)};
      float r[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) r[q] = bf2f(mh[q]) > 0.f ? acc[mb][nb][q] : 0.f;
      *(uint2*)(out + o) = make_uint2(pk_bf16(r[0], r[1]), pk_bf16(r[2], r[3]));
    }
  }
}

// Weight and bias gradients of one layer: dW[o][tap][i] = sum over pixels of
// dy[p][o] x[p + tap offset][i], as a GEMM with M = output channels, N = 9
// taps x input channels (padded to 16), K = pixels, on
// v_mfma_f32_16x16x32_bf16 (operand layout as in k_conv).  A workgroup stages the transposed dy of
// an 8 x 32 block and three column-shifted, channel-major copies of the input
// patch (so that four consecutive pixels of an operand are one aligned 8-byte
// read), loops over `bpw` blocks, then adds its partial sums atomically.
//   CINM / CINR: input channels in memory / real; DYC: dy channels in memory;
//   COUTP / COUTR: output channels padded to 16 / real.
template <int CINM, int CINR, int DYC, int COUTP, int COUTR>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ x,
                                               const uint16_t* __restrict__ dy,
                                               float* __restrict__ part, int N, int H, int W, int bpw) {
  constexpr int KN = kpad16(CINM), MB = COUTP / 16, NB = KN / 16;
  constexpr int NW = COUTR * 9 * CINR;     // weights of the layer; its COUTR biases follow
  constexpr int PR = BH + 2;
  // wave w computes the 16-column blocks nb = w, w + 4, ... of the result for
  // every 16-channel block mb: one x operand read serves MB products
  constexpr int PER_WAVE = (NB + 3) / 4;
  static_assert(MB <= 2, "at most 32 output channels");
  // Row strides padded by 8 values: unpadded (512 and 640 bytes) the 16 rows
  // of one operand read started on 1 or 2 distinct 16-byte bank groups (16-
  // and 8-fold conflicts); 528 and 656 bytes spread them over all 16.
  constexpr int DS = BH * BW + 8;          // dyt: one output channel
  constexpr int XS = PR * BW + 8;          // xs: one (column shift, input channel) plane
  __shared__ __align__(16) uint16_t dyt[COUTP * DS];
  __shared__ __align__(16) uint16_t xs[3 * CINM * XS];
  const int nbx = (W + BW - 1) / BW, nby = (H + BH - 1) / BH, nblocks = nbx * nby * N;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, i16 = lane & 15, g4 = lane >> 4;
  f4 acc[PER_WAVE][MB];
#pragma unroll
  for (int k = 0; k < PER_WAVE; ++k)
#pragma unroll
    for (int m = 0; m < MB; ++m) acc[k][m] = f4{0.f, 0.f, 0.f, 0.f};
  // bias gradient: per-thread partial sums of the dy channels this thread
  // loads (channels 8 (tid & 3) .. + 7 for 32-channel dy, 0 .. 3 for 4)
  float bpart[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) bpart[j] = 0.f;
  if constexpr (DYC == 4) {
    // rows of the output channels beyond the four in memory stay zero
    for (int idx = 4 * DS + tid; idx < COUTP * DS; idx += 256) dyt[idx] = 0;
  }
  for (int bi = 0; bi < bpw; ++bi) {
    const int blk = blockIdx.x * bpw + bi;
    if (blk >= nblocks) break;
    const int bx = blk % nbx, by = (blk / nbx) % nby, n = blk / (nbx * nby);
    // Every global read of the block is issued first, into registers (while
    // the previous block's products may still read LDS), and the LDS writes
    // follow: the staging waits for memory once per block instead of once per
    // loop iteration.
    // dy: 16-byte (8-channel) or 8-byte (4-channel) pixel pieces, zero outside
    // the image, two horizontally adjacent pixels per item
    constexpr int DYI = DYC == 32 ? BH * BW / 2 * 4 : BH * BW / 2, NDY = (DYI + 255) / 256;
    uint4 dv[NDY][2];
#pragma unroll
    for (int it = 0; it < NDY; ++it) {
      const int idx = tid + 256 * it;
      const int pp = DYC == 32 ? idx >> 2 : idx, ch = DYC == 32 ? idx & 3 : 0;
      const int gy = by * BH + (2 * pp) / BW;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int gx = bx * BW + (2 * pp) % BW + hh;
        dv[it][hh] = make_uint4(0u, 0u, 0u, 0u);
        if (idx < DYI && gy < H && gx < W) {
          if constexpr (DYC == 32) {
            dv[it][hh] = *(const uint4*)(dy + ((size_t)(n * H + gy) * W + gx) * 32 + ch * 8);
          } else {
            const uint2 v = *(const uint2*)(dy + ((size_t)(n * H + gy) * W + gx) * 4);
            dv[it][hh] = make_uint4(v.x, v.y, 0u, 0u);
          }
        }
      }
    }
    // x: the patch of the block grown by one pixel (34 columns), the same
    // pieces, two horizontally adjacent pixels per item
    constexpr int XC = CINM == 32 ? 4 : 1;     // 16- or 8-byte pieces per pixel
    constexpr int NPR = (BW + 2) / 2;          // column pairs per patch row
    constexpr int XI = PR * NPR * XC, NXI = (XI + 255) / 256;
    uint4 xv[NXI][2];
#pragma unroll
    for (int it = 0; it < NXI; ++it) {
      const int idx = tid + 256 * it;
      const int q = idx / XC, ch = idx - q * XC;
      const int r = q / NPR, m = q - r * NPR;
      const int gy = by * BH + r - 1;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int gx = bx * BW + 2 * m + hh - 1;
        xv[it][hh] = make_uint4(0u, 0u, 0u, 0u);
        if (idx < XI && gy >= 0 && gy < H && gx >= 0 && gx < W) {
          if constexpr (CINM == 32) {
            xv[it][hh] = *(const uint4*)(x + ((size_t)(n * H + gy) * W + gx) * 32 + ch * 8);
          } else {
            const uint2 v = *(const uint2*)(x + ((size_t)(n * H + gy) * W + gx) * 4);
            xv[it][hh] = make_uint4(v.x, v.y, 0u, 0u);
          }
        }
      }
    }
    __syncthreads();   // the previous block's reads of dyt and xs are done
    // dy transposed, dyt[o][r * 32 + c], a 4-byte word per pixel pair
#pragma unroll
    for (int it = 0; it < NDY; ++it) {
      const int idx = tid + 256 * it;
      if (idx >= DYI) break;
      const int pp = DYC == 32 ? idx >> 2 : idx, ch = DYC == 32 ? idx & 3 : 0;
      const uint32_t w0[4] = {dv[it][0].x, dv[it][0].y, dv[it][0].z, dv[it][0].w};
      const uint32_t w1[4] = {dv[it][1].x, dv[it][1].y, dv[it][1].z, dv[it][1].w};
#pragma unroll
      for (int j = 0; j < (DYC == 32 ? 8 : 4); ++j) {
        const bool real = DYC == 32 || j < COUTR;
        const uint32_t h0 = real ? (w0[j >> 1] >> (16 * (j & 1))) & 0xffffu : 0u;
        const uint32_t h1 = real ? (w1[j >> 1] >> (16 * (j & 1))) & 0xffffu : 0u;
        *(uint32_t*)(dyt + (ch * 8 + j) * DS + 2 * pp) = h0 | (h1 << 16);
        bpart[j] += bf2f((uint16_t)h0) + bf2f((uint16_t)h1);
      }
    }
    // xs[kx][i][r][c] = x[by*8 + r - 1][bx*32 + c + kx - 1][i]: each pair of
    // patch columns (2m, 2m + 1) goes to the copies whose column range holds
    // it -- as one 4-byte word in copies 0 and 2 (columns 2m and 2m - 2 there,
    // even), as two halves in copy 1
#pragma unroll
    for (int it = 0; it < NXI; ++it) {
      const int idx = tid + 256 * it;
      if (idx >= XI) break;
      const int q = idx / XC, ch = idx - q * XC;
      const int r = q / NPR, m = q - r * NPR;
      const uint32_t w0[4] = {xv[it][0].x, xv[it][0].y, xv[it][0].z, xv[it][0].w};
      const uint32_t w1[4] = {xv[it][1].x, xv[it][1].y, xv[it][1].z, xv[it][1].w};
#pragma unroll
      for (int j = 0; j < (CINM == 32 ? 8 : 4); ++j) {
        const uint32_t h0 = (w0[j >> 1] >> (16 * (j & 1))) & 0xffffu;
        const uint32_t h1 = (w1[j >> 1] >> (16 * (j & 1))) & 0xffffu;
        const int i = ch * 8 + j, row = r * BW + 2 * m;
        if (m < NPR - 1) {
          *(uint32_t*)(xs + i * XS + row) = h0 | (h1 << 16);
          xs[(CINM + i) * XS + row] = (uint16_t)h1;
        }
        if (m > 0) {
          *(uint32_t*)(xs + (2 * CINM + i) * XS + row - 2) = h0 | (h1 << 16);
          xs[(CINM + i) * XS + row - 1] = (uint16_t)h0;
        }
      }
    }
    __syncthreads();
    // K steps of 32 pixels: one block row each, lane group g4 taking
    // columns 8 g4 .. 8 g4 + 7 of both operands
#pragma unroll 1
    for (int row = 0; row < BH; ++row) {
      const int c0 = g4 * 8;
      // the dy operand of each 16-channel block, read once per row
      bf8 a[MB];
#pragma unroll
      for (int m = 0; m < MB; ++m) a[m] = as_bf8(*(const uint4*)(dyt + (m * 16 + i16) * DS + row * BW + c0));
#pragma unroll
      for (int k = 0; k < PER_WAVE; ++k) {
        const int nb = wave + 4 * k;
        if (nb >= NB) break;
        const int nn = nb * 16 + i16, tap = nn / CINM, i = nn - tap * CINM;
        uint4 bx4 = make_uint4(0u, 0u, 0u, 0u);
        if (tap < 9) {
          const int ky = tap / 3, kx = tap - ky * 3;
          bx4 = *(const uint4*)(xs + (kx * CINM + i) * XS + (row + ky) * BW + c0);
        }
#pragma unroll
        for (int m = 0; m < MB; ++m)
          acc[k][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], as_bf8(bx4), acc[k][m], 0, 0, 0);
      }
    }
  }
  // this workgroup's partial sums, plain stores into its row of `part`
  // (parameter layout: dW, then db); k_wsum adds the rows up
  float* row_out = part + (size_t)blockIdx.x * (NW + COUTR);
#pragma unroll
  for (int k = 0; k < PER_WAVE; ++k) {
    const int nb = wave + 4 * k;
    if (nb >= NB) break;
    const int nn = nb * 16 + i16, tap = nn / CINM, i = nn - tap * CINM;
    if (tap >= 9 || i >= CINR) continue;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = m * 16 + g4 * 4 + q;
        if (o < COUTR) row_out[(o * 9 + tap) * CINR + i] = acc[k][m][q];
      }
  }
  // bias gradient: lanes holding the same channels, then the four waves
  __shared__ float bred[4][32];
  if constexpr (DYC == 32) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int m = 4; m < 64; m <<= 1) bpart[j] += __shfl_xor(bpart[j], m);
    if (lane < 4)
#pragma unroll
      for (int j = 0; j < 8; ++j) bred[wave][lane * 8 + j] = bpart[j];
  } else {
#pragma unroll
    for (int j = 0; j < COUTR; ++j)
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) bpart[j] += __shfl_xor(bpart[j], m);
    if (lane == 0)
#pragma unroll
      for (int j = 0; j < COUTR; ++j) bred[wave][j] = bpart[j];
  }
  __syncthreads();
  if (tid < COUTR) row_out[NW + tid] = bred[0][tid] + bred[1][tid] + bred[2][tid] + bred[3][tid];
}

// Sum of the weight-gradient kernel's per-workgroup rows into the gradient
// (zeroed before): thread j of column block x adds rows 32 y .. 32 y + 31 of
// parameter j, one atomic per 32 rows.
__global__ __launch_bounds__(256) void k_wsum(const float* __restrict__ part, int rows, int width,
                                              float* __restrict__ g) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= width) return;
  const int r0 = blockIdx.y * 32, r1 = min(r0 + 32, rows);
  float s = 0.f;
#pragma unroll 8
  for (int r = r0; r < r1; ++r) s += part[(size_t)r * width + j];
  atomicAdd(&g[j], s);
}

// The whole forward pass in one kernel (3 -> 32 -> 32 -> 32 -> 3): a
// workgroup computes a 16 x 32 output tile and keeps every intermediate
// activation on chip.  Each layer is computed on the region the next one
// needs -- the tile grown by one pixel per remaining layer (22 x 38, 20 x 36,
// 18 x 34 pixels) -- so that no activation is read back from memory; pixels
// of a region outside the image are zero, the padding every layer applies.
// The four weight matrices (50 KB of bf16) and the image patch are staged in
// LDS once; each layer's matrix is then copied into registers by every wave.
// The MFMA operand layout and K order are k_conv's (above); activations are
// rounded to bfloat16 after the ReLU, as the backward pass reads them.  KEEP:
// also write the three ReLU activations of the tile's own pixels to memory
// for the backward pass.  Sixteen waves (four per SIMD) hide the LDS and
// barrier latencies of the one workgroup that fits a CU.
constexpr int FH = 16, FW = 32;                       // output tile
constexpr int FWAVES = 16;                            // waves per workgroup (four per SIMD)
constexpr int kW1 = 32 * 64, kW2 = 32 * 288, kW4 = 16 * 288;
constexpr int kWAll = kW1 + 2 * kW2 + kW4;            // bf16 weights of the four layers

struct FwdArgs {
  const uint16_t* w[4];    // bf16 weights, [coutp][kpad32(cin)]
  const float* b[4];       // fp32 biases
  uint16_t* act[3];        // ReLU outputs, [pixels][32] (KEEP)
};

// One layer from LDS region `in` to region `out` (LI = 1..3) or to z (LI = 4).
// Regions are row-major pixel arrays; 32-channel ones are four planes of
// 8-channel (16-byte) pixels with a stride of PIN / POUT entries.
template <int LI, bool KEEP>
__device__ __forceinline__ void fwd_layer(const void* in, uint4* out, const uint16_t* wl, const float* __restrict__ bias,
                                          uint16_t* __restrict__ act, float* __restrict__ z, int n, int H, int W,
                                          int y0, int x0, int wave, int lane) {
  constexpr int CIN = LI == 1 ? 4 : 32, COUT = LI == 4 ? 16 : 32, NB = COUT / 16;
  constexpr int KP = kpad32(CIN), KS = KP / 32;
  constexpr int GROW = 4 - LI;                             // output region: tile grown by GROW
  constexpr int HO = FH + 2 * GROW, WO = FW + 2 * GROW, WI = WO + 2;
  constexpr int NPX = HO * WO, NPB = (NPX + 15) / 16;
  constexpr int PIN = (HO + 2) * WI + 1, POUT = NPX + 1;   // plane strides (32-channel regions)
  // every 16-pixel block of the wave in one pass: G blocks, computed without
  // a branch (blocks past the region read clamped pixels and are dropped at
  // the end), so that each K step's LDS reads go out together
  constexpr int G = (NPB + FWAVES - 1) / FWAVES;
  const int i16 = lane & 15, g = lane >> 4;
  const int oy0 = y0 - GROW, ox0 = x0 - GROW;               // image position of the region's origin

  bf8 wr[KS][NB];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) wr[ks][nb] = as_bf8(*(const uint4*)(wl + (nb * 16 + i16) * KP + ks * 32 + 8 * g));
  float bv[NB][4];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int co = nb * 16 + 4 * g + q;
      bv[nb][q] = (LI < 4 || co < 3) ? bias[co] : 0.f;
    }

  for (int pb0 = wave; pb0 < NPB; pb0 += FWAVES * G) {
    f4 acc[G][NB];
    int pix[G], src[G];
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
      pix[gi] = (pb0 + FWAVES * gi) * 16 + i16;
      const int pc = min(pix[gi], NPX - 1), oy = pc / WO, ox = pc - oy * WO;
      src[gi] = oy * WI + ox;                                 // input pixel of tap (0, 0)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[gi][nb] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      uint4 bqs[G];
#pragma unroll
      for (int gi = 0; gi < G; ++gi) {
        uint4 bq;
        if constexpr (CIN == 32) {
          const int ky = ks / 3, kx = ks - 3 * (ks / 3);
          bq = ((const uint4*)in)[g * PIN + src[gi] + ky * WI + kx];
        } else {
          const uint2* p8 = (const uint2*)in;
          const int t0 = ks * 8 + 2 * g, t1 = t0 + 1;
          const int u0 = min(t0, 8), u1 = min(t1, 8);
          uint2 lo = p8[src[gi] + (u0 / 3) * WI + u0 % 3];
          uint2 hi = p8[src[gi] + (u1 / 3) * WI + u1 % 3];
          if (t0 >= 9) lo = make_uint2(0u, 0u);
          if (t1 >= 9) hi = make_uint2(0u, 0u);
          bq = make_uint4(lo.x, lo.y, hi.x, hi.y);
        }
        bqs[gi] = bq;
      }
#pragma unroll
      for (int gi = 0; gi < G; ++gi) {
        const bf8 b = as_bf8(bqs[gi]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[gi][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[ks][nb], b, acc[gi][nb], 0, 0, 0);
      }
    }
    // epilogue: lane (g, i16) holds channels nb * 16 + 4 g .. + 3 of pixel pix
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
      if (pb0 + FWAVES * gi >= NPB) break;
      const int p = pix[gi];
      if (p >= NPX) continue;
      const int oy = p / WO, ox = p - oy * WO, gy = oy0 + oy, gx = ox0 + ox;
      const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
      if constexpr (LI == 4) {
        if (g == 0 && inside)
          *(float4*)(z + ((size_t)(n * H + gy) * W + gx) * 4) =
              make_float4(acc[gi][0][0] + bv[0][0], acc[gi][0][1] + bv[0][1], acc[gi][0][2] + bv[0][2], 0.f);
      } else {
        const bool keep = KEEP && inside && oy >= GROW && oy < GROW + FH && ox >= GROW && ox < GROW + FW;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          float r[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) r[q] = inside ? fmaxf(acc[gi][nb][q] + bv[nb][q], 0.f) : 0.f;
          const uint2 v = make_uint2(pk_bf16(r[0], r[1]), pk_bf16(r[2], r[3]));
          ((uint2*)out)[((2 * nb + (g >> 1)) * POUT + p) * 2 + (g & 1)] = v;
          if (keep) *(uint2*)(act + ((size_t)(n * H + gy) * W + gx) * 32 + nb * 16 + 4 * g) = v;
        }
      }
    }
  }
}

template <bool KEEP>
__global__ __launch_bounds__(64 * FWAVES) void k_forward(const uint16_t* __restrict__ x, const FwdArgs fa,
                                                 float* __restrict__ z, int N, int H, int W) {
  constexpr int R0W = FW + 8, R0H = FH + 8;
  constexpr int PA = (FH + 6) * (FW + 6) + 1, PB = (FH + 4) * (FW + 4) + 1;
  __shared__ __align__(16) uint16_t wl[kWAll];
  __shared__ __align__(16) uint2 r0[R0H * R0W];
  __shared__ __align__(16) uint4 ra[4 * PA];     // layer 1's output, then layer 3's
  __shared__ __align__(16) uint4 rb[4 * PB];     // layer 2's output
  const int nbx = (W + FW - 1) / FW, nby = (H + FH - 1) / FH;
  const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, n = blockIdx.x / (nbx * nby);
  const int y0 = by * FH, x0 = bx * FW;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // the four weight matrices, one after the other
  for (int i = tid; i < kWAll / 8; i += 64 * FWAVES) {
    const int e = i * 8;
    const uint16_t* src = e < kW1 ? fa.w[0] + e
                        : e < kW1 + kW2 ? fa.w[1] + (e - kW1)
                        : e < kW1 + 2 * kW2 ? fa.w[2] + (e - kW1 - kW2)
                        : fa.w[3] + (e - kW1 - 2 * kW2);
    *(uint4*)(wl + e) = *(const uint4*)src;
  }
  // the image patch: the tile grown by four pixels, zero outside the image
  for (int p = tid; p < R0H * R0W; p += 64 * FWAVES) {
    const int r = p / R0W, c = p - r * R0W;
    const int gy = y0 - 4 + r, gx = x0 - 4 + c;
    uint2 v = make_uint2(0u, 0u);
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = *(const uint2*)(x + ((size_t)(n * H + gy) * W + gx) * 4);
    r0[p] = v;
  }
  __syncthreads();
  fwd_layer<1, KEEP>(r0, ra, wl, fa.b[0], fa.act[0], z, n, H, W, y0, x0, wave, lane);
  __syncthreads();
  fwd_layer<2, KEEP>(ra, rb, wl + kW1, fa.b[1], fa.act[1], z, n, H, W, y0, x0, wave, lane);
  __syncthreads();
  fwd_layer<3, KEEP>(rb, ra, wl + kW1 + kW2, fa.b[2], fa.act[2], z, n, H, W, y0, x0, wave, lane);
  __syncthreads();
  fwd_layer<4, KEEP>(ra, nullptr, wl + kW1 + 2 * kW2, fa.b[3], nullptr, z, n, H, W, y0, x0, wave, lane);
}

// MSE of y = x + z against t (three channels): dL/dz = 2 (y - t) / count as
// bfloat16, and the mean squared difference accumulated into *loss.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ z, const uint16_t* __restrict__ x,
                                              const float* __restrict__ t, uint16_t* __restrict__ dz,
                                              float* __restrict__ loss, int P, float scale,
                                              float inv_count) {
  __shared__ float red[256];
  const int p = blockIdx.x * 256 + threadIdx.x;
  float s = 0.f;
  if (p < P) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      float d = 0.f;
      if (c < 3) {
        d = bf2f(x[p * 4 + c]) + z[p * 4 + c] - t[p * 4 + c];
        s += d * d;
      }
      dz[p * 4 + c] = f2bf(scale * d);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] * inv_count);
}

// Adam on the fp32 parameters.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Parameter layout (fp32): per layer, W[out][3][3][in] then b[out].
struct Layer {
  int cinr, coutr, cinm, coutp;   // real / memory input channels, real / padded output channels
  int w_off, b_off;               // offsets in the parameter vector
};
constexpr int kLayers = 4;

// bfloat16 weights for the forward convolutions ([coutp][kpad32(cinm)], zero
// padded) and, for layers 1..3, for the backward convolutions: the kernel
// flipped and transposed, W'[i][2-ky][2-kx][o] = W[o][ky][kx][i], laid out
// for a convolution from the layer's output channels to its input channels.
__device__ __forceinline__ void prep_one(const float* __restrict__ params, uint16_t* __restrict__ wf,
                                         uint16_t* __restrict__ wb, const Layer& L, bool is_fwd, int idx) {
  if (is_fwd) {
    const int KP = kpad32(L.cinm);
    if (idx >= L.coutp * KP) return;
    const int o = idx / KP, k = idx - o * KP, tap = k / L.cinm, i = k - tap * L.cinm;
    float v = 0.f;
    if (o < L.coutr && tap < 9 && i < L.cinr) v = params[L.w_off + (o * 9 + tap) * L.cinr + i];
    wf[idx] = f2bf(v);
  } else {
    // backward conv: input channels = this layer's outputs (in memory: 4 or 32),
    // output channels = this layer's inputs (32)
    const int cin2 = L.coutr == 3 ? 4 : L.coutr, KP = kpad32(cin2);
    if (idx >= HID * KP) return;
    const int o2 = idx / KP, k = idx - o2 * KP, tap2 = k / cin2, i2 = k - tap2 * cin2;
    float v = 0.f;
    if (tap2 < 9 && i2 < L.coutr && o2 < L.cinr) {
      const int ky = 2 - tap2 / 3, kx = 2 - tap2 % 3;
      v = params[L.w_off + (i2 * 9 + ky * 3 + kx) * L.cinr + o2];
    }
    wb[idx] = f2bf(v);
  }
}

// Every layer's forward and backward matrices in one launch: segment k < 4
// is layer k's forward matrix, segment 4 + k its backward one (empty for
// layer 0); start[] holds each segment's first index.
struct PrepArgs {
  Layer L[kLayers];
  uint16_t* wf[kLayers];
  uint16_t* wb[kLayers];
  int start[2 * kLayers + 1];
};

__global__ void k_prep(const float* __restrict__ params, const PrepArgs a) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.start[2 * kLayers]) return;
  int seg = 0;
#pragma unroll
  for (int k = 1; k < 2 * kLayers; ++k)
    if (idx >= a.start[k]) seg = k;
  const int li = seg % kLayers;
  const bool fwd = seg < kLayers;
  prep_one(params, a.wf[li], a.wb[li], a.L[li], fwd, idx - a.start[seg]);
}

// Images (tile-planar uint8 RGB viewports, [V][ty*tx][3][T][T]) to network
// tensors: crops (v, y0, x0) of S x S as bfloat16 NHWC4 in [0, 1] (or fp32).
__global__ void k_gather(const uint8_t* __restrict__ img, int T, int tx, int ty,
                         const int* __restrict__ crops, int S, void* __restrict__ out, int as_float) {
  const int b = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= S * S) return;
  const int v = crops[3 * b], y = crops[3 * b + 1] + p / S, xg = crops[3 * b + 2] + p % S;
  const size_t tile = (size_t)v * tx * ty + (y / T) * tx + xg / T;
  const size_t base = tile * 3 * T * T + (size_t)(y % T) * T + xg % T;
  const size_t o = ((size_t)b * S * S + p) * 4;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float f = c < 3 ? img[base + (size_t)c * T * T] * (1.f / 255.f) : 0.f;
    if (as_float)
      ((float*)out)[o + c] = f;
    else
      ((uint16_t*)out)[o + c] = f2bf(f);
  }
}

// A whole tile-planar viewport (ty x tx tiles of T x T) as one bfloat16
// NHWC4 image in [0, 1].
__global__ void k_to_nhwc(const uint8_t* __restrict__ img, int T, int tx, int ty,
                          uint16_t* __restrict__ out) {
  const int W = T * tx;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= W * T * ty) return;
  const int y = p / W, xg = p % W;
  const size_t base = ((size_t)(y / T) * tx + xg / T) * 3 * T * T + (size_t)(y % T) * T + xg % T;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    out[(size_t)p * 4 + c] = c < 3 ? f2bf(img[base + (size_t)c * T * T] * (1.f / 255.f)) : (uint16_t)0;
}

// Per-tile guard statistics of a restored viewport: sum of |z| and a count
// of non-finite values, per T x T tile.  One workgroup per (tile, band of
// `rows` rows) sums its pixels and adds once per tile: per-pixel atomics on
// one address per tile serialise in the cache and took milliseconds.
__global__ __launch_bounds__(256) void k_guard(const float* __restrict__ z, int T, int tx, int rows,
                                               float* __restrict__ absz, int* __restrict__ bad) {
  const int W = T * tx;
  const int tile = blockIdx.x, tyi = tile / tx, txi = tile - tyi * tx;
  const int r0 = blockIdx.y * rows, r1 = min(r0 + rows, T);
  float s = 0.f;
  int nb = 0;
  for (int i = threadIdx.x; i < (r1 - r0) * T; i += 256) {
    const int r = r0 + i / T, c = i - (i / T) * T;
    const size_t p = (size_t)(tyi * T + r) * W + txi * T + c;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float v = z[p * 4 + ch];
      if (!isfinite(v)) ++nb;
      else s += fabsf(v);
    }
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    s += __shfl_xor(s, m);
    nb += __shfl_xor(nb, m);
  }
  __shared__ float rs[4];
  __shared__ int rn[4];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rs[wave] = s;
    rn[wave] = nb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&absz[tile], rs[0] + rs[1] + rs[2] + rs[3]);
    const int n = rn[0] + rn[1] + rn[2] + rn[3];
    if (n) atomicAdd(&bad[tile], n);
  }
}

// Restored viewport: clip(x + z) in 8 bits, or the decoded tile where the
// guard tripped.
__global__ void k_restore(const uint8_t* __restrict__ dec, const float* __restrict__ z, int T, int tx,
                          int ty, const int* __restrict__ use, uint8_t* __restrict__ out) {
  const int W = T * tx;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= W * T * ty) return;
  const int y = p / W, xg = p % W;
  const int tile = (y / T) * tx + xg / T;
  const size_t base = (size_t)tile * 3 * T * T + (size_t)(y % T) * T + xg % T;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const uint8_t d = dec[base + (size_t)c * T * T];
    uint8_t o = d;
    if (use[tile]) {
      const float f = d * (1.f / 255.f) + z[(size_t)p * 4 + c];
      o = (uint8_t)fminf(fmaxf(rintf(f * 255.f), 0.f), 255.f);
    }
    out[base + (size_t)c * T * T] = o;
  }
}

}  // namespace cnn
}  // namespace wv

using namespace wv;
using namespace wv::cnn;
using wvp::fail;
using wvp::hip_fail;

// weight gradients: at most this many workgroups, each writing one row of
// partial sums
constexpr int kWgradRows = 512;

struct wv_cnn {
  Layer layer[kLayers];
  int n_params = 0;
  int64_t max_pixels = 0;
  float* params = nullptr;     // fp32 masters
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t* wf[kLayers] = {};   // forward bfloat16 weights
  uint16_t* wb[kLayers] = {};   // backward bfloat16 weights (layers 1..3)
  uint16_t* x = nullptr;        // [P][4] input buffer (restore writes its viewport here)
  const uint16_t* xin = nullptr;  // input of the last forward, read in place
  float* zout = nullptr;        // output of the last forward
  uint16_t* act[3] = {};        // [P][32]
  uint16_t* dbuf[2] = {};       // [P][32]
  float* z = nullptr;           // [P][4]
  uint16_t* dz = nullptr;       // [P][4]
  float* loss = nullptr;        // device scalar
  float* guard_abs = nullptr;   // per-tile guard sums
  int* guard_bad = nullptr;
  int* guard_use = nullptr;
  int* crops = nullptr;
  float* wpart = nullptr;       // weight-gradient partial sums, [kWgradRows][largest layer]
  int n = 0, h = 0, w = 0;      // shape of the last forward
  bool fwd_valid = false, grad_valid = false;
  bool prepped = false;
};

static void layer_table(Layer* L, int& total) {
  const int cinr[kLayers] = {3, HID, HID, HID}, coutr[kLayers] = {HID, HID, HID, 3};
  int off = 0;
  for (int i = 0; i < kLayers; ++i) {
    L[i].cinr = cinr[i];
    L[i].coutr = coutr[i];
    L[i].cinm = cinr[i] == 3 ? 4 : cinr[i];
    L[i].coutp = coutr[i] == 3 ? 16 : coutr[i];
    L[i].w_off = off;
    off += coutr[i] * 9 * cinr[i];
    L[i].b_off = off;
    off += coutr[i];
  }
  total = off;
}

extern "C" int32_t wv_cnn_param_count(void) {
  Layer L[kLayers];
  int t = 0;
  layer_table(L, t);
  return t;
}

extern "C" wv_status wv_cnn_destroy(wv_cnn* net) {
  if (!net) return WV_OK;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {net->params, net->grads, net->adam_m, net->adam_v, net->x, net->act[0], net->act[1],
                  net->act[2], net->dbuf[0], net->dbuf[1], net->z, net->dz, net->loss, net->guard_abs,
                  net->guard_bad, net->guard_use, net->crops, net->wpart};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int i = 0; i < kLayers; ++i) {
    if (net->wf[i]) (void)hipFree(net->wf[i]);
    if (net->wb[i]) (void)hipFree(net->wb[i]);
  }
  delete net;
  return WV_OK;
}

extern "C" wv_status wv_cnn_create(wv_cnn** out, int64_t max_pixels) {
  if (!out || max_pixels < 1 || max_pixels > ((int64_t)1 << 28))
    return fail(WV_EINVAL, "wv_cnn_create: max_pixels must be 1 .. 2^28");
  *out = nullptr;
  wv_cnn* net = new (std::nothrow) wv_cnn();
  if (!net) return fail(WV_ENOMEM, "wv_cnn allocation");
  layer_table(net->layer, net->n_params);
  net->max_pixels = max_pixels;
  const size_t P = (size_t)max_pixels, np = (size_t)net->n_params * sizeof(float);
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
    if (e == hipSuccess) e = hipMemset(*p, 0, bytes);
  };
  alloc((void**)&net->params, np);
  alloc((void**)&net->grads, np);
  alloc((void**)&net->adam_m, np);
  alloc((void**)&net->adam_v, np);
  for (int i = 0; i < kLayers; ++i) {
    alloc((void**)&net->wf[i], (size_t)net->layer[i].coutp * kpad32(net->layer[i].cinm) * 2);
    if (i > 0) alloc((void**)&net->wb[i], (size_t)HID * kpad32(net->layer[i].coutr == 3 ? 4 : HID) * 2);
  }
  alloc((void**)&net->x, P * 4 * 2);
  for (int i = 0; i < 3; ++i) alloc((void**)&net->act[i], P * HID * 2);
  for (int i = 0; i < 2; ++i) alloc((void**)&net->dbuf[i], P * HID * 2);
  alloc((void**)&net->z, P * 4 * 4);
  alloc((void**)&net->dz, P * 4 * 2);
  alloc((void**)&net->loss, sizeof(float));
  alloc((void**)&net->guard_abs, 65536 * sizeof(float));
  alloc((void**)&net->guard_bad, 65536 * sizeof(int));
  alloc((void**)&net->guard_use, 65536 * sizeof(int));
  alloc((void**)&net->crops, 3 * 4096 * sizeof(int));
  alloc((void**)&net->wpart, (size_t)kWgradRows * (HID * 9 * HID + HID) * sizeof(float));
  if (e != hipSuccess) {
    wv_cnn_destroy(net);
    return e == hipErrorOutOfMemory ? fail(WV_ENOMEM, "wv_cnn buffers: %s", hipGetErrorString(e))
                                    : hip_fail(e, "wv_cnn_create");
  }
  *out = net;
  return WV_OK;
}

static wv_status prep(wv_cnn* net, hipStream_t s) {
  PrepArgs a;
  int at = 0;
  for (int i = 0; i < kLayers; ++i) {
    const Layer& L = net->layer[i];
    a.L[i] = L;
    a.wf[i] = net->wf[i];
    a.wb[i] = net->wb[i];
    a.start[i] = at;
    at += L.coutp * kpad32(L.cinm);
  }
  for (int i = 0; i < kLayers; ++i) {
    const Layer& L = net->layer[i];
    a.start[kLayers + i] = at;
    if (i > 0) at += HID * kpad32(L.coutr == 3 ? 4 : HID);
  }
  a.start[2 * kLayers] = at;
  hipLaunchKernelGGL(k_prep, dim3((at + 255) / 256), dim3(256), 0, s, net->params, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "wv_cnn weight preparation");
  net->prepped = true;
  return WV_OK;
}

extern "C" wv_status wv_cnn_set_params(wv_cnn* net, const float* host_params, hipStream_t s) {
  if (!net || !host_params) return fail(WV_EINVAL, "wv_cnn_set_params: bad argument");
  hipError_t e = hipMemcpyAsync(net->params, host_params, (size_t)net->n_params * 4,
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(net->adam_m, 0, (size_t)net->n_params * 4, s);
  if (e == hipSuccess) e = hipMemsetAsync(net->adam_v, 0, (size_t)net->n_params * 4, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "wv_cnn_set_params");
  return prep(net, s);
}

extern "C" wv_status wv_cnn_get_params(wv_cnn* net, float* host_params, hipStream_t s) {
  if (!net || !host_params) return fail(WV_EINVAL, "wv_cnn_get_params: bad argument");
  hipError_t e = hipMemcpyAsync(host_params, net->params, (size_t)net->n_params * 4,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? WV_OK : hip_fail(e, "wv_cnn_get_params");
}

static int conv_grid(int n, int h, int w) { return n * ((h + CH - 1) / CH) * ((w + CW - 1) / CW); }
static int wgrad_blocks(int n, int h, int w) { return n * ((h + BH - 1) / BH) * ((w + BW - 1) / BW); }

// The forward pass in one launch; keep: write the activations the backward
// pass reads.
static wv_status forward(wv_cnn* net, const uint16_t* x, int32_t n, int32_t h, int32_t w, float* z, bool keep,
                         hipStream_t s) {
  const char* fn = keep ? "wv_cnn_forward" : "wv_cnn_infer";
  if (!net || !x || n < 1 || h < 1 || w < 1) return fail(WV_EINVAL, "%s: bad argument", fn);
  if ((int64_t)n * h * w > net->max_pixels)
    return fail(WV_EINVAL, "%s: %lld pixels above the %lld the network was created for", fn,
                (long long)n * h * w, (long long)net->max_pixels);
  if (!net->prepped) return fail(WV_EINVAL, "%s: parameters not set", fn);
  float* zo = z ? z : net->z;
  const Layer* L = net->layer;
  FwdArgs fa;
  for (int i = 0; i < kLayers; ++i) {
    fa.w[i] = net->wf[i];
    fa.b[i] = net->params + L[i].b_off;
  }
  for (int i = 0; i < 3; ++i) fa.act[i] = net->act[i];
  const dim3 g(conv_grid(n, h, w)), b(64 * FWAVES);
  if (keep)
    hipLaunchKernelGGL(k_forward<true>, g, b, 0, s, x, fa, zo, n, h, w);
  else
    hipLaunchKernelGGL(k_forward<false>, g, b, 0, s, x, fa, zo, n, h, w);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, fn);
  net->xin = x;
  net->zout = zo;
  net->n = n;
  net->h = h;
  net->w = w;
  net->fwd_valid = keep;
  net->grad_valid = false;
  return WV_OK;
}

extern "C" wv_status wv_cnn_forward(wv_cnn* net, const uint16_t* x, int32_t n, int32_t h, int32_t w,
                                    float* z, hipStream_t s) {
  return forward(net, x, n, h, w, z, true, s);
}

extern "C" wv_status wv_cnn_infer(wv_cnn* net, const uint16_t* x, int32_t n, int32_t h, int32_t w, float* z,
                                  hipStream_t s) {
  return forward(net, x, n, h, w, z, false, s);
}

extern "C" wv_status wv_cnn_loss_grad(wv_cnn* net, const float* t, float* loss, hipStream_t s) {
  if (!net || !t || !loss) return fail(WV_EINVAL, "wv_cnn_loss_grad: bad argument");
  if (!net->fwd_valid) return fail(WV_EINVAL, "wv_cnn_loss_grad: no forward pass to differentiate");
  const int P = net->n * net->h * net->w;
  hipError_t e = hipMemsetAsync(net->loss, 0, sizeof(float), s);
  if (e != hipSuccess) return hip_fail(e, "wv_cnn_loss_grad");
  hipLaunchKernelGGL(k_loss, dim3((P + 255) / 256), dim3(256), 0, s, net->zout, net->xin, t, net->dz,
                     net->loss, P, 2.0f / (3.0f * (float)P), 1.0f / (3.0f * (float)P));
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(loss, net->loss, sizeof(float), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "wv_cnn_loss_grad");
  net->grad_valid = true;
  return WV_OK;
}

extern "C" wv_status wv_cnn_backward(wv_cnn* net, float* grads, hipStream_t s) {
  if (!net) return fail(WV_EINVAL, "wv_cnn_backward: bad argument");
  if (!net->grad_valid) return fail(WV_EINVAL, "wv_cnn_backward: no loss gradient");
  const int n = net->n, h = net->h, w = net->w;
  const Layer* L = net->layer;
  hipError_t e = hipMemsetAsync(net->grads, 0, (size_t)net->n_params * 4, s);
  if (e != hipSuccess) return hip_fail(e, "wv_cnn_backward");
  const dim3 g(conv_grid(n, h, w)), b(256);
  const int nblocks = wgrad_blocks(n, h, w);
  // split over pixels: at most kWgradRows workgroups, each writing a row of
  // partial sums that k_wsum adds into the gradient
  const int bpw = (nblocks + kWgradRows - 1) / kWgradRows;
  const int rows = (nblocks + bpw - 1) / bpw;
  const dim3 gw(rows);
  auto wsum = [&](const Layer& l) {
    const int width = l.coutr * 9 * l.cinr + l.coutr;
    hipLaunchKernelGGL(k_wsum, dim3((width + 255) / 256, (rows + 31) / 32), b, 0, s, (const float*)net->wpart,
                       rows, width, net->grads + l.w_off);
  };
  // layer 4: dW4 from a3 and dz; d3 = (W4' * dz) masked by a3 > 0
  hipLaunchKernelGGL((k_wgrad<HID, HID, 4, 16, 3>), gw, b, 0, s, net->act[2], net->dz, net->wpart, n, h, w, bpw);
  wsum(L[3]);
  hipLaunchKernelGGL((k_conv<4, HID>), g, b, 0, s, net->dz, net->wb[3], net->act[2], net->dbuf[0], n, h, w);
  // layer 3
  hipLaunchKernelGGL((k_wgrad<HID, HID, HID, HID, HID>), gw, b, 0, s, net->act[1], net->dbuf[0], net->wpart,
                     n, h, w, bpw);
  wsum(L[2]);
  hipLaunchKernelGGL((k_conv<HID, HID>), g, b, 0, s, net->dbuf[0], net->wb[2], net->act[1], net->dbuf[1], n, h,
                     w);
  // layer 2
  hipLaunchKernelGGL((k_wgrad<HID, HID, HID, HID, HID>), gw, b, 0, s, net->act[0], net->dbuf[1], net->wpart,
                     n, h, w, bpw);
  wsum(L[1]);
  hipLaunchKernelGGL((k_conv<HID, HID>), g, b, 0, s, net->dbuf[1], net->wb[1], net->act[0], net->dbuf[0], n, h,
                     w);
  // layer 1
  hipLaunchKernelGGL((k_wgrad<4, 3, HID, HID, HID>), gw, b, 0, s, net->xin, net->dbuf[0], net->wpart, n, h, w,
                     bpw);
  wsum(L[0]);
  e = hipGetLastError();
  if (e == hipSuccess && grads && grads != net->grads)
    e = hipMemcpyAsync(grads, net->grads, (size_t)net->n_params * 4, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "wv_cnn_backward");
  return WV_OK;
}

extern "C" wv_status wv_cnn_adam(wv_cnn* net, float lr, int32_t step, hipStream_t s) {
  if (!net || step < 1 || !(lr > 0)) return fail(WV_EINVAL, "wv_cnn_adam: bad argument");
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((net->n_params + 255) / 256), dim3(256), 0, s, net->params, net->grads,
                     net->adam_m, net->adam_v, net->n_params, lr, b1, b2, 1e-8f, c1, c2);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "wv_cnn_adam");
  return prep(net, s);
}

extern "C" wv_status wv_cnn_train_step(wv_cnn* net, const uint16_t* x, const float* t, int32_t n,
                                       int32_t h, int32_t w, float lr, int32_t step, float* loss,
                                       hipStream_t s) {
  wv_status st = wv_cnn_forward(net, x, n, h, w, nullptr, s);
  if (st == WV_OK) st = wv_cnn_loss_grad(net, t, loss, s);
  if (st == WV_OK) st = wv_cnn_backward(net, nullptr, s);
  if (st == WV_OK) st = wv_cnn_adam(net, lr, step, s);
  return st;
}

extern "C" wv_status wv_cnn_gather(wv_cnn* net, const uint8_t* images, int32_t tile, int32_t tiles_x,
                                   int32_t tiles_y, int32_t n_images, const int32_t* crops,
                                   int32_t n_crops, int32_t size, int32_t as_float, void* out,
                                   hipStream_t s) {
  if (!net || !images || !crops || !out || tile < 1 || tiles_x < 1 || tiles_y < 1 || n_crops < 1 ||
      n_crops > 4096 || size < 1)
    return fail(WV_EINVAL, "wv_cnn_gather: bad argument");
  for (int i = 0; i < n_crops; ++i) {
    const int v = crops[3 * i], y0 = crops[3 * i + 1], x0 = crops[3 * i + 2];
    if (v < 0 || v >= n_images || y0 < 0 || x0 < 0 || y0 + size > tile * tiles_y ||
        x0 + size > tile * tiles_x)
      return fail(WV_EINVAL, "wv_cnn_gather: crop %d outside its image", i);
  }
  // the crop table is copied synchronously: the network's table buffer is
  // reused by the next call
  hipError_t e = hipMemcpyAsync(net->crops, crops, (size_t)n_crops * 3 * sizeof(int),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gather, dim3((size * size + 255) / 256, n_crops), dim3(256), 0, s, images, tile,
                       tiles_x, tiles_y, (const int*)net->crops, size, out, as_float);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? WV_OK : hip_fail(e, "wv_cnn_gather");
}

extern "C" wv_status wv_cnn_restore(wv_cnn* net, const uint8_t* decoded, int32_t tile, int32_t tiles_x,
                                    int32_t tiles_y, float guard, uint8_t* out, int32_t* fallback_tiles,
                                    hipStream_t s) {
  if (!net || !decoded || !out || tile < 1 || tiles_x < 1 || tiles_y < 1 || !(guard > 0))
    return fail(WV_EINVAL, "wv_cnn_restore: bad argument");
  const int nt = tiles_x * tiles_y;
  if (nt > 65536) return fail(WV_EINVAL, "wv_cnn_restore: at most 65536 tiles");
  const int H = tile * tiles_y, W = tile * tiles_x;
  if ((int64_t)H * W > net->max_pixels) return fail(WV_EINVAL, "wv_cnn_restore: image above max_pixels");
  const int P = H * W, gb = (P + 255) / 256;
  // the input goes straight into the network's input buffer
  hipLaunchKernelGGL(k_to_nhwc, dim3(gb), dim3(256), 0, s, decoded, tile, tiles_x, tiles_y, net->x);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "wv_cnn_restore");
  // inference only: the activations are not needed
  wv_status st = forward(net, net->x, 1, H, W, nullptr, false, s);
  if (st != WV_OK) return st;
  e = hipMemsetAsync(net->guard_abs, 0, nt * sizeof(float), s);
  if (e == hipSuccess) e = hipMemsetAsync(net->guard_bad, 0, nt * sizeof(int), s);
  if (e == hipSuccess) {
    const int rows = std::max(1, 4096 / tile);
    hipLaunchKernelGGL(k_guard, dim3(nt, (tile + rows - 1) / rows), dim3(256), 0, s, net->z, tile, tiles_x, rows,
                       net->guard_abs, net->guard_bad);
    e = hipGetLastError();
  }
  std::vector<float> absz(nt);
  std::vector<int> bad(nt), use(nt);
  if (e == hipSuccess) e = hipMemcpyAsync(absz.data(), net->guard_abs, nt * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(bad.data(), net->guard_bad, nt * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "wv_cnn_restore guard");
  // guard: a tile keeps the network's output only if every value is finite
  // and its mean correction (0..1 scale) stays below `guard`
  int fell = 0;
  const double per_tile = 3.0 * tile * tile;
  for (int i = 0; i < nt; ++i) {
    use[i] = bad[i] == 0 && absz[i] / per_tile <= guard;
    fell += !use[i];
  }
  e = hipMemcpyAsync(net->guard_use, use.data(), nt * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_restore, dim3(gb), dim3(256), 0, s, decoded, net->z, tile, tiles_x, tiles_y,
                       (const int*)net->guard_use, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "wv_cnn_restore");
  if (fallback_tiles) *fallback_tiles = fell;
  return WV_OK;
}
