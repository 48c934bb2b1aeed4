// Row-strip fused decode kernels for the 5/3 wavelet, frames of inter-frame sets.
#include "wv_strip_launch.h"

namespace wv {

hipError_t launch_strip53_set(int format, int shape, int L, const WorkArgs& a, hipStream_t s) {
  return strip::launch<Inv53, true>(format, shape, L, false, a, 0, s);
}

}  // namespace wv
