// Feature detection areas of a rig (Alg. 2, step 1; Sec. 4.1): the part of each frame
// where, after the cameras' rough alignment, a neighbouring frame overlaps it.  Host-only:
// no HIP call.
//
// Camera i's footprint F_i is the bounding box of its frame rectangle's corners (0, 0),
// (w, 0), (w, h), (0, h) mapped by H_i (source -> canvas).  For every pair i < j whose
// footprints overlap with positive area, the overlap widened by `margin` canvas pixels on
// every side and clipped to the canvas, O_ij, is mapped back into each frame of the pair
// through adj(H_k) (H_k^-1 up to scale); the bounding box of O_ij's four corner images,
// rounded outward with a slack of 1e-6 sample and clipped to the frame, is one detection
// area of frame k (if it is not empty).  A frame's areas come in the order of the partner
// camera.  A footprint (or a corner image) is bounded only when the projective depth has
// one sign, never zero, at the four corners; a camera whose footprint is unbounded gets
// no areas, and an overlap whose corner images are unbounded in frame k gives frame k
// its whole rectangle.
#include <algorithm>
#include <cmath>

#include "stitch.h"
#include "stitch_internal.h"

using namespace stitch;

namespace {

constexpr double kSlack = 1e-6;

struct Box {
  double x0, y0, x1, y1;
};

// Images of the four corners of `b` under the 3x3 row-major map m, as a bounding box;
// false when the depth does not keep one sign or a coordinate is not finite.
bool map_box(const double* m, const Box& b, Box* out) {
#pragma clang fp contract(off)
  const double xs[4] = {b.x0, b.x1, b.x1, b.x0};
  const double ys[4] = {b.y0, b.y0, b.y1, b.y1};
  double z0 = 0.0;
  Box r{1e300, 1e300, -1e300, -1e300};
  for (int c = 0; c < 4; ++c) {
    const double z = m[6] * xs[c] + m[7] * ys[c] + m[8];
    if (!(z != 0.0) || !std::isfinite(z)) return false;
    if (c == 0) z0 = z;
    else if ((z > 0.0) != (z0 > 0.0)) return false;
    const double X = (m[0] * xs[c] + m[1] * ys[c] + m[2]) / z;
    const double Y = (m[3] * xs[c] + m[4] * ys[c] + m[5]) / z;
    if (!std::isfinite(X) || !std::isfinite(Y)) return false;
    r.x0 = std::min(r.x0, X); r.x1 = std::max(r.x1, X);
    r.y0 = std::min(r.y0, Y); r.y1 = std::max(r.y1, Y);
  }
  *out = r;
  return true;
}

// adj(H): H^-1 up to a non-zero scale (which the projective division removes).
void adjugate(const double* a, double* adj) {
#pragma clang fp contract(off)
  adj[0] = a[4] * a[8] - a[5] * a[7];
  adj[1] = a[2] * a[7] - a[1] * a[8];
  adj[2] = a[1] * a[5] - a[2] * a[4];
  adj[3] = a[5] * a[6] - a[3] * a[8];
  adj[4] = a[0] * a[8] - a[2] * a[6];
  adj[5] = a[2] * a[3] - a[0] * a[5];
  adj[6] = a[3] * a[7] - a[4] * a[6];
  adj[7] = a[1] * a[6] - a[0] * a[7];
  adj[8] = a[0] * a[4] - a[1] * a[3];
}

}  // namespace

extern "C" stitch_status stitch_detection_areas(int32_t n, const int32_t* frame_w, const int32_t* frame_h,
                                                const double* H, int32_t canvas_w, int32_t canvas_h,
                                                int32_t margin, int32_t max_areas, int32_t* counts,
                                                int32_t* areas) {
  if (!frame_w || !frame_h || !H || !counts || !areas)
    return fail(STITCH_E_NULL, "frame_w, frame_h, H, counts or areas is NULL");
  if (n < 1 || n > kMaxCameras) return fail(STITCH_E_SHAPE, "n = %d outside 1..%d", n, kMaxCameras);
  if (canvas_w < 1 || canvas_h < 1 || canvas_w > (1 << 20) || canvas_h > (1 << 20))
    return fail(STITCH_E_SHAPE, "canvas %dx%d outside 1..2^20", canvas_w, canvas_h);
  if (margin < 0 || margin > (1 << 20)) return fail(STITCH_E_SHAPE, "margin %d outside 0..2^20", margin);
  if (max_areas < 1) return fail(STITCH_E_SHAPE, "max_areas %d < 1", max_areas);
  for (int i = 0; i < n; ++i) {
    if (frame_w[i] < 1 || frame_h[i] < 1 || frame_w[i] > (1 << 20) || frame_h[i] > (1 << 20))
      return fail(STITCH_E_SHAPE, "frame %d has size %dx%d (sides 1 .. 2^20)", i, frame_w[i], frame_h[i]);
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(H[9 * i + k])) return fail(STITCH_E_HOMOGRAPHY, "H of camera %d has a non-finite entry", i);
  }
  Box F[kMaxCameras];
  bool bounded[kMaxCameras];
  double adj[kMaxCameras][9];
  for (int i = 0; i < n; ++i) {
    bounded[i] = map_box(H + 9 * i, Box{0.0, 0.0, (double)frame_w[i], (double)frame_h[i]}, &F[i]);
    adjugate(H + 9 * i, adj[i]);
    counts[i] = 0;
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      if (!bounded[i] || !bounded[j]) continue;
      Box o{std::max(F[i].x0, F[j].x0), std::max(F[i].y0, F[j].y0), std::min(F[i].x1, F[j].x1),
            std::min(F[i].y1, F[j].y1)};
      if (!(o.x1 > o.x0 && o.y1 > o.y0)) continue;
      o.x0 = std::max(o.x0 - margin, 0.0);
      o.y0 = std::max(o.y0 - margin, 0.0);
      o.x1 = std::min(o.x1 + margin, (double)canvas_w);
      o.y1 = std::min(o.y1 + margin, (double)canvas_h);
      if (!(o.x1 > o.x0 && o.y1 > o.y0)) continue;
      for (const int k : {i, j}) {
        Box f;
        const double w = frame_w[k], h = frame_h[k];
        int64_t x0 = 0, y0 = 0, x1 = frame_w[k], y1 = frame_h[k];
        if (map_box(adj[k], o, &f)) {
          x0 = std::max<int64_t>(0, (int64_t)std::max(-1.0, std::floor(f.x0 - kSlack)));
          y0 = std::max<int64_t>(0, (int64_t)std::max(-1.0, std::floor(f.y0 - kSlack)));
          x1 = std::min<int64_t>(frame_w[k], (int64_t)std::min(w + 1.0, std::ceil(f.x1 + kSlack)));
          y1 = std::min<int64_t>(frame_h[k], (int64_t)std::min(h + 1.0, std::ceil(f.y1 + kSlack)));
        }
        if (x1 <= x0 || y1 <= y0) continue;
        if (counts[k] >= max_areas)
          return fail(STITCH_E_SHAPE, "frame %d has more than max_areas = %d areas", k, max_areas);
        int32_t* a = areas + ((int64_t)k * max_areas + counts[k]) * 4;
        a[0] = (int32_t)x0; a[1] = (int32_t)y0; a[2] = (int32_t)(x1 - x0); a[3] = (int32_t)(y1 - y0);
        ++counts[k];
      }
    }
  return STITCH_OK;
}
