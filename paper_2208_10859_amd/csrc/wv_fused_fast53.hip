// Fast fused decode kernels for the 5/3 wavelet (compile-time level counts 3, 4, 5).
#include "wv_fused_fast.h"

namespace wv {

template <class LF, int FMT, int L>
static hipError_t launch_fast_l(int shape, bool pers, const WorkArgs& a, int n_cu, hipStream_t s) {
#define WV_FAST(bw, bh, tr, gpc)                                                              \
  {                                                                                         \
    const int grid = pers ? min(a.total, n_cu * (gpc)) : a.total;                           \
    if (grid <= 0) return hipSuccess;                                                       \
    if (pers)                                                                               \
      hipLaunchKernelGGL((k_fused_fast<LF, FMT, bw, bh, tr, L, true>), dim3(grid),          \
                         dim3((bw / 2) * (bh / tr)), 0, s, a);                              \
    else                                                                                    \
      hipLaunchKernelGGL((k_fused_fast<LF, FMT, bw, bh, tr, L, false>), dim3(grid),         \
                         dim3((bw / 2) * (bh / tr)), 0, s, a);                              \
    return hipGetLastError();                                                               \
  }
  switch (shape) {
    case 0: WV_FAST(64, 64, 8, 4)
    case 1: WV_FAST(64, 128, 16, 3)
    case 2: WV_FAST(128, 32, 8, 4)
  }
#undef WV_FAST
  return hipErrorInvalidValue;
}

template <class LF, int FMT>
static hipError_t launch_fast_f(int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                                hipStream_t s) {
  switch (L) {
    case 3: return launch_fast_l<LF, FMT, 3>(shape, pers, a, n_cu, s);
    case 4: return launch_fast_l<LF, FMT, 4>(shape, pers, a, n_cu, s);
    case 5: return launch_fast_l<LF, FMT, 5>(shape, pers, a, n_cu, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fast53(int format, int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                         hipStream_t s) {
  return format == WV_YUV420 ? launch_fast_f<Inv53, WV_YUV420>(shape, L, pers, a, n_cu, s)
                             : launch_fast_f<Inv53, WV_GRAY8>(shape, L, pers, a, n_cu, s);
}

}  // namespace wv
