// Rebuild of dense coefficient planes from the sparse storage format
// (Section 3.5's GPU rebuild of the wavelet image from uploaded records).
//
// One workgroup per (visible tile, block): the block is assembled in LDS --
// zeroed, then every record of the block dequantised (Eq. 4 inverted) and
// placed at its index -- and written to the dense plane in coalesced rows.
// Blocks of levels the tile's level count drops are skipped whole.
#include <hip/hip_runtime.h>

#include "wv_internal.h"

namespace wv {

// Eq. 4 inverted: c = lo + code * scale with the product and the sum each
// rounded to float32.  Contraction is off here: HIP's __fmul_rn / __fadd_rn
// are plain operators that the compiler would fuse into one FMA, which rounds
// once and gives a different value.
__device__ __forceinline__ float dequantise(float code, float lo, float scale) {
#pragma clang fp contract(off)
  return lo + code * scale;
}

template <class OUT>
__device__ __forceinline__ OUT to_dense(float v);
template <>
__device__ __forceinline__ float to_dense<float>(float v) { return v; }
template <>
__device__ __forceinline__ int16_t to_dense<int16_t>(float v) {
  return (int16_t)fminf(fmaxf(__builtin_rintf(v), -32768.0f), 32767.0f);
}

template <class OUT>
__global__ __launch_bounds__(256) void k_rebuild(const RebuildArgs a) {
  __shared__ __attribute__((aligned(16))) OUT blk[32 * 32];
  const int item = blockIdx.x / a.nb, j = blockIdx.x - item * a.nb;
  const Item it = a.items[item];
  const int by = a.order[j] >> 8, bx = a.order[j] & 0xff;
  const int b = a.b, p = a.p, levels = a.levels;
  // level of the block: that of the detail region its origin lies in
  const int m = max(by, bx) * b;
  int lev = levels + 1;
  for (int k = levels; k >= 1; --k)
    if (m >= (p >> k)) lev = k;
  if (lev <= levels - (int)it.lc) return;   // a dropped level: not read
  // block ends of the whole plane are indexed by tile; staged ones (only the
  // visible tiles, in output order) by the item's slot
  const uint64_t g = (uint64_t)(a.compact ? it.slot : it.tile) * a.nb + j;
  uint64_t s = g ? a.block_end[g - 1] : 0, e = a.block_end[g];
  s = min(s, a.n_records);
  e = min(max(e, s), a.n_records);
  const int nbb = b * b, tid = threadIdx.x;
  // each thread's first record is read before the block is zeroed (the read
  // then overlaps the zeroing and its barrier); blocks rarely hold more
  // records than threads
  const uint64_t r0 = s + tid;
  int idx0 = nbb;
  uint8_t val0 = 0;
  if (r0 < e) {
    idx0 = a.index[r0];
    val0 = a.values[r0];
  }
  // zero the block: 16 bytes per thread
  constexpr int V16 = 16 / sizeof(OUT);
  for (int i = tid * V16; i < nbb; i += 256 * V16) *(int4*)&blk[i] = make_int4(0, 0, 0, 0);
  __syncthreads();
  const int ap = p >> levels;                // edge of the approximation band
  auto place = [&](int idx, uint8_t code) {
    if (idx >= nbb) return;
    const int y = by * b + idx / b, x = bx * b + idx % b;
    const int cls = (y < ap && x < ap) ? 0 : 1;
    blk[idx] = to_dense<OUT>(dequantise((float)code, a.lo[cls], a.scale[cls]));
  };
  place(idx0, val0);
  for (uint64_t r = r0 + 256; r < e; r += 256) place(a.index[r], a.values[r]);
  __syncthreads();
  OUT* dst = (OUT*)a.dense + (size_t)it.tile * p * p + (size_t)(by * b) * p + bx * b;
  if (b == 32) {
    // 32 rows of 32 values: 8 threads per row, 4 values each (a 16-byte
    // store for float32, 8 bytes for int16)
    const int yy = tid >> 3, xx = (tid & 7) * 4;
    if constexpr (sizeof(OUT) == 4)
      *(int4*)(dst + (size_t)yy * p + xx) = *(const int4*)&blk[yy * 32 + xx];
    else
      *(int2*)(dst + (size_t)yy * p + xx) = *(const int2*)&blk[yy * 32 + xx];
  } else {
    for (int i = tid; i < nbb; i += 256) {
      const int yy = i / b, xx = i - yy * b;
      dst[(size_t)yy * p + xx] = blk[i];
    }
  }
}

hipError_t launch_rebuild(int wavelet, const RebuildArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  const dim3 grid(a.n_items * a.nb);
  if (wavelet == WV_W53)
    hipLaunchKernelGGL(k_rebuild<int16_t>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_rebuild<float>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace wv
