// Row-strip fused decode kernels for the 5/3 wavelet.
#include "wv_strip.h"

namespace wv {

template <class LF, int FMT, int L, int R, int NW, int GPC, int WPE, int WPEP, int SCHED>
static hipError_t launch_one(bool pers, const WorkArgs& a, int n_cu, hipStream_t s) {
  const int grid = pers ? min(a.total, n_cu * GPC) : a.total;
  if (grid <= 0) return hipSuccess;
  if (pers) {
    if constexpr (GPC > 0)
      hipLaunchKernelGGL((strip::k_strip<LF, FMT, 512, L, R, NW, true, WPEP, SCHED>), dim3(grid),
                         dim3(64 * NW), 0, s, a);
    else
      return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((strip::k_strip<LF, FMT, 512, L, R, NW, false, WPE, SCHED>), dim3(grid),
                       dim3(64 * NW), 0, s, a);
  }
  return hipGetLastError();
}

// Shapes: strip rows, waves, persistent groups per CU (0: grid form only),
// waves per SIMD to leave register room for (grid form, persistent form).
template <class LF, int FMT, int L>
static hipError_t launch_strip_l(int shape, bool pers, const WorkArgs& a, int n_cu, hipStream_t s) {
  switch (shape) {
    case 0: return launch_one<LF, FMT, L, 32, 4, 2, 3, 2, 0>(pers, a, n_cu, s);
    case 1: return launch_one<LF, FMT, L, 16, 4, 3, 4, 3, 0>(pers, a, n_cu, s);
    case 2: return launch_one<LF, FMT, L, 32, 8, 0, 4, 4, 0>(pers, a, n_cu, s);
    case 3: return launch_one<LF, FMT, L, 32, 4, 0, 3, 3, 1>(pers, a, n_cu, s);
    case 4: return launch_one<LF, FMT, L, 16, 4, 0, 4, 4, 1>(pers, a, n_cu, s);
  }
  return hipErrorInvalidValue;
}

template <class LF, int FMT>
static hipError_t launch_strip_f(int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                                 hipStream_t s) {
  switch (L) {
    case 3: return launch_strip_l<LF, FMT, 3>(shape, pers, a, n_cu, s);
    case 4: return launch_strip_l<LF, FMT, 4>(shape, pers, a, n_cu, s);
    case 5: return launch_strip_l<LF, FMT, 5>(shape, pers, a, n_cu, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_strip53(int format, int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                          hipStream_t s) {
  return format == WV_YUV420 ? launch_strip_f<Inv53, WV_YUV420>(shape, L, pers, a, n_cu, s)
                             : launch_strip_f<Inv53, WV_GRAY8>(shape, L, pers, a, n_cu, s);
}

}  // namespace wv
