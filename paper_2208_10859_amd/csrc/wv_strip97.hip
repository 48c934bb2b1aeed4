// Row-strip fused decode kernels for the 9/7 wavelet, stored frames.
#include "wv_strip_launch.h"

namespace wv {

hipError_t launch_strip97(int format, int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                          hipStream_t s) {
  return strip::launch<Inv97, false>(format, shape, L, pers, a, n_cu, s);
}

}  // namespace wv
