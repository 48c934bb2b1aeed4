// Viewport tile selection and foveated level counts (host, float64).
//
// The mask is defined on a coarse version of the frame (one entry per tile)
// and is independent of the mapping (Sections 3.1 and 3.6); the geometry here
// is the equirectangular, top-bottom stereo one: each eye is a width x
// height/2 image, longitude -180..180 degrees left to right, latitude
// 90..-90 degrees top to bottom.  A tile is selected when one of its sample
// points maps to a direction inside the rectilinear frustum around the head
// direction.  Foveation (Section 3.7) keeps all levels near the gaze and
// drops the finest one or two levels with growing eccentricity.
#include <cmath>

#include "wv.h"
#include "wv_geom.h"

using namespace wvg;

namespace {

bool desc_ok(const wv_desc* d) {
  return d && d->tile > 0 && d->width > 0 && d->height > 0 && d->width % d->tile == 0 &&
         d->height % d->tile == 0;
}

}  // namespace

extern "C" wv_status wv_viewport_mask(const wv_desc* d, double yaw, double pitch, double fov_h,
                                      double fov_v, int32_t samples, int32_t eyes,
                                      uint8_t* mask) {
  if (!desc_ok(d) || !mask || samples < 1 || (eyes != 1 && eyes != 2) || !(fov_h > 0.0) ||
      !(fov_h < 180.0) || !(fov_v > 0.0) || !(fov_v < 180.0))
    return WV_EINVAL;
  const int ntx = d->width / d->tile, nty = d->height / d->tile;
  const double eye_h = d->height / 2.0;
  const Camera c = camera(yaw, pitch);
  const double th = std::tan(fov_h * (M_PI / 360.0)), tv = std::tan(fov_v * (M_PI / 360.0));
  for (int ty = 0; ty < nty; ++ty) {
    const int eye = tile_eye(ty, d->tile, eye_h);
    for (int tx = 0; tx < ntx; ++tx) {
      uint8_t hit = 0;
      if (eye < eyes) {
        for (int i = 0; i < samples && !hit; ++i)
          for (int j = 0; j < samples && !hit; ++j) {
            double dir[3];
            sample_direction(tx, ty, i, j, d->tile, samples, (double)d->width, eye_h, dir);
            if (in_frustum(dir, c, th, tv)) hit = 1;
          }
      }
      mask[ty * ntx + tx] = hit;
    }
  }
  return WV_OK;
}

extern "C" wv_status wv_foveation_levels(const wv_desc* d, double yaw, double pitch, double inner,
                                         double outer, uint8_t* level_count) {
  if (!desc_ok(d) || !level_count || d->levels < 0 || !(inner >= 0.0) || !(outer >= inner))
    return WV_EINVAL;
  const int ntx = d->width / d->tile, nty = d->height / d->tile;
  const double eye_h = d->height / 2.0;
  const Camera c = camera(yaw, pitch);
  for (int ty = 0; ty < nty; ++ty)
    for (int tx = 0; tx < ntx; ++tx) {
      double dir[3];
      centre_direction(tx, ty, d->tile, (double)d->width, eye_h, dir);
      level_count[ty * ntx + tx] =
          (uint8_t)foveated_levels(d->levels, eccentricity(dir, c), inner, outer);
    }
  return WV_OK;
}
