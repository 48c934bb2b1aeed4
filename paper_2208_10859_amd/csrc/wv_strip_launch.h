// Launchers of the row-strip kernels.  Each wavelet's kernels are compiled
// in two translation units: stored frames, and inter-frame-set frames (SET),
// whose coefficients are summed from three temporal bands at load time.
#pragma once
#include "wv_strip.h"

namespace wv {
namespace strip {

template <class LF, int FMT, int L, int R, int NW, int GPC, int WPE, int WPEP, int SCHED, bool SET>
static hipError_t launch_one(bool pers, const WorkArgs& a, int n_cu, hipStream_t s) {
  const int grid = pers ? min(a.total, n_cu * GPC) : a.total;
  if (grid <= 0) return hipSuccess;
  if (pers) {
    if constexpr (GPC > 0 && !SET)
      hipLaunchKernelGGL((k_strip<LF, FMT, 512, L, R, NW, true, WPEP, SCHED, SET>), dim3(grid),
                         dim3(64 * NW), 0, s, a);
    else
      return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((k_strip<LF, FMT, 512, L, R, NW, false, WPE, SCHED, SET>), dim3(grid),
                       dim3(64 * NW), 0, s, a);
  }
  return hipGetLastError();
}

// Shapes: strip rows, waves, persistent groups per CU (0: grid form only),
// waves per SIMD to leave register room for (grid form, persistent form);
// the 9/7 lifting state needs more registers than the 5/3 one.  Set frames
// run the grid form only; the 8-wave shape runs as the 4-wave one.
template <class LF, int FMT, int L, bool SET>
static hipError_t launch_shape(int shape, bool pers, const WorkArgs& a, int n_cu, hipStream_t s) {
  constexpr bool W53 = std::is_same<LF, Inv53>::value;
  // grey 9/7 set frames at 16 rows: three band loads per value need the
  // register room of two waves per SIMD
  constexpr int W97R16 = SET && FMT == WV_GRAY8 ? 2 : 3;
  if constexpr (SET) {
    if (shape == 2) shape = 0;
    pers = false;
  }
  switch (shape) {
    case 0: return launch_one<LF, FMT, L, 32, 4, 2, W53 ? 3 : 2, 2, 0, SET>(pers, a, n_cu, s);
    case 1: return launch_one<LF, FMT, L, 16, 4, W53 ? 3 : 2, W53 ? 4 : W97R16, W53 ? 3 : 2, 0, SET>(pers, a, n_cu, s);
    case 2:
      if constexpr (!SET) return launch_one<LF, FMT, L, 32, 8, 0, W53 ? 4 : 3, W53 ? 4 : 3, 0, SET>(pers, a, n_cu, s);
      break;
    case 3: return launch_one<LF, FMT, L, 32, 4, 0, W53 ? 3 : 2, W53 ? 3 : 2, 1, SET>(pers, a, n_cu, s);
    // 16-row chain units use 29.7 KB of LDS (YUV420): five fit on a CU, and
    // the stored-frame 5/3 kernel fits the registers of five waves per SIMD
    case 4: return launch_one<LF, FMT, L, 16, 4, W53 ? 5 : 3, W53 ? (SET ? 4 : 5) : W97R16, W53 ? 5 : 3, 1, SET>(pers, a, n_cu, s);
  }
  return hipErrorInvalidValue;
}

template <class LF, bool SET>
static hipError_t launch(int format, int shape, int L, bool pers, const WorkArgs& a, int n_cu,
                         hipStream_t s) {
  if (format == WV_YUV420) {
    switch (L) {
      case 3: return launch_shape<LF, WV_YUV420, 3, SET>(shape, pers, a, n_cu, s);
      case 4: return launch_shape<LF, WV_YUV420, 4, SET>(shape, pers, a, n_cu, s);
      case 5: return launch_shape<LF, WV_YUV420, 5, SET>(shape, pers, a, n_cu, s);
    }
  } else {
    switch (L) {
      case 3: return launch_shape<LF, WV_GRAY8, 3, SET>(shape, pers, a, n_cu, s);
      case 4: return launch_shape<LF, WV_GRAY8, 4, SET>(shape, pers, a, n_cu, s);
      case 5: return launch_shape<LF, WV_GRAY8, 5, SET>(shape, pers, a, n_cu, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace strip
}  // namespace wv
