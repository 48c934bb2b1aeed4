// Row-strip fused decode kernels for the 9/7 wavelet, frames of inter-frame sets.
#include "wv_strip_launch.h"

namespace wv {

hipError_t launch_strip97_set(int format, int shape, int L, const WorkArgs& a, hipStream_t s) {
  return strip::launch<Inv97, true>(format, shape, L, false, a, 0, s);
}

}  // namespace wv
