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

namespace {

struct Camera {
  double f[3], r[3], u[3];
};

// Head frame for yaw p, pitch t (radians): forward, right, up.
Camera camera(double yaw_deg, double pitch_deg) {
  const double p = yaw_deg * (M_PI / 180.0), t = pitch_deg * (M_PI / 180.0);
  Camera c;
  c.f[0] = std::cos(t) * std::sin(p);
  c.f[1] = std::sin(t);
  c.f[2] = std::cos(t) * std::cos(p);
  c.r[0] = std::cos(p);
  c.r[1] = 0.0;
  c.r[2] = -std::sin(p);
  c.u[0] = -std::sin(t) * std::sin(p);
  c.u[1] = std::cos(t);
  c.u[2] = -std::sin(t) * std::cos(p);
  return c;
}

// Unit direction of the equirectangular position (x, y) in an eye image.
void direction(double x, double y, double eye_w, double eye_h, double d[3]) {
  const double lon = (x / eye_w) * (2.0 * M_PI) - M_PI;
  const double lat = 0.5 * M_PI - (y / eye_h) * M_PI;
  const double cl = std::cos(lat);
  d[0] = cl * std::sin(lon);
  d[1] = std::sin(lat);
  d[2] = cl * std::cos(lon);
}

double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

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
    const int eye = (double)(ty * d->tile) < eye_h ? 0 : 1;
    for (int tx = 0; tx < ntx; ++tx) {
      uint8_t hit = 0;
      if (eye < eyes) {
        for (int i = 0; i < samples && !hit; ++i) {
          const double y = ty * d->tile + (i + 0.5) * ((double)d->tile / samples) - eye * eye_h;
          for (int j = 0; j < samples && !hit; ++j) {
            const double x = tx * d->tile + (j + 0.5) * ((double)d->tile / samples);
            double dir[3];
            direction(x, y, (double)d->width, eye_h, dir);
            const double zf = dot(dir, c.f), xr = dot(dir, c.r), yu = dot(dir, c.u);
            if (zf > 0.0 && std::fabs(xr) <= th * zf && std::fabs(yu) <= tv * zf) hit = 1;
          }
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
  for (int ty = 0; ty < nty; ++ty) {
    const int eye = (double)(ty * d->tile) < eye_h ? 0 : 1;
    for (int tx = 0; tx < ntx; ++tx) {
      double dir[3];
      direction((tx + 0.5) * d->tile, (ty + 0.5) * d->tile - eye * eye_h, (double)d->width, eye_h,
                dir);
      const double cs = std::fmax(-1.0, std::fmin(1.0, dot(dir, c.f)));
      const double ecc = std::acos(cs) * (180.0 / M_PI);
      const int drop = ecc <= inner ? 0 : (ecc <= outer ? 1 : 2);
      level_count[ty * ntx + tx] = (uint8_t)(d->levels > drop ? d->levels - drop : 0);
    }
  }
  return WV_OK;
}
