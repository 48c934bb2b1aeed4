// Private to libwv: viewing geometry shared by the public selection calls
// and the serving loop (host, float64).  Each eye of the top-bottom stereo
// frame is an equirectangular width x height/2 image: longitude -180..180
// degrees left to right, latitude 90..-90 degrees top to bottom.
#pragma once

#include <cmath>

namespace wvg {

struct Camera {
  double f[3], r[3], u[3];   // forward, right, up
};

// Head frame for yaw and pitch in degrees.
inline Camera camera(double yaw_deg, double pitch_deg) {
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
inline void direction(double x, double y, double eye_w, double eye_h, double d[3]) {
  const double lon = (x / eye_w) * (2.0 * M_PI) - M_PI;
  const double lat = 0.5 * M_PI - (y / eye_h) * M_PI;
  const double cl = std::cos(lat);
  d[0] = cl * std::sin(lon);
  d[1] = std::sin(lat);
  d[2] = cl * std::cos(lon);
}

inline double dot(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Eye (0 top, 1 bottom) of tile row ty.
inline int tile_eye(int ty, int tile, double eye_h) { return (double)(ty * tile) < eye_h ? 0 : 1; }

// Direction of sample (i, j) of samples x samples inside tile (tx, ty).
inline void sample_direction(int tx, int ty, int i, int j, int tile, int samples, double width,
                             double eye_h, double d[3]) {
  const int eye = tile_eye(ty, tile, eye_h);
  const double y = ty * tile + (i + 0.5) * ((double)tile / samples) - eye * eye_h;
  const double x = tx * tile + (j + 0.5) * ((double)tile / samples);
  direction(x, y, width, eye_h, d);
}

// Direction of the centre of tile (tx, ty).
inline void centre_direction(int tx, int ty, int tile, double width, double eye_h, double d[3]) {
  const int eye = tile_eye(ty, tile, eye_h);
  direction((tx + 0.5) * tile, (ty + 0.5) * tile - eye * eye_h, width, eye_h, d);
}

// Inside the rectilinear frustum of half-extents tan th, tan tv.
inline bool in_frustum(const double d[3], const Camera& c, double th, double tv) {
  const double zf = dot(d, c.f), xr = dot(d, c.r), yu = dot(d, c.u);
  return zf > 0.0 && std::fabs(xr) <= th * zf && std::fabs(yu) <= tv * zf;
}

// Eccentricity (degrees) of a direction from the gaze.
inline double eccentricity(const double d[3], const Camera& c) {
  const double cs = std::fmax(-1.0, std::fmin(1.0, dot(d, c.f)));
  return std::acos(cs) * (180.0 / M_PI);
}

// Levels applied at an eccentricity: all within inner degrees, one fewer
// within outer degrees, two fewer beyond (never below zero).
inline int foveated_levels(int levels, double ecc, double inner, double outer) {
  const int drop = ecc <= inner ? 0 : (ecc <= outer ? 1 : 2);
  return levels > drop ? levels - drop : 0;
}

}  // namespace wvg
