"""Plain CPU oracle of the feature detection areas (Sec. 4.1, Alg. 2 step 1).

TEST INFRASTRUCTURE ONLY: tests/ and bench.py may import it; the HIP product path never
does, and the two share no code, header, table or helper.

The paper reduces L-ORB's detection to the parts of each frame that the neighbouring
frames overlap once the cameras are roughly aligned, without fixing how the overlap is
measured.  Reading R37 (numbered after the registration readings R27-R36):

  R37 camera i's footprint is the axis-aligned bounding box of the images under H_i
      (source -> canvas) of its frame rectangle's corners (0, 0), (w, 0), (w, h), (0, h);
      it is bounded only when the projective depth keeps one sign, never zero, at the
      four corners (otherwise the camera gets no areas).  For every pair i < j whose
      footprints overlap with positive area, the overlap is widened by `margin` canvas
      pixels on every side and clipped to the canvas [0, W] x [0, H]; its four corners are
      mapped into frame k (k = i, j) by the inverse of H_k, and the bounding box of those
      images, rounded outward with a slack of 1e-6 sample ([floor(min - 1e-6),
      ceil(max + 1e-6))) and clipped to [0, w_k) x [0, h_k), is an area of frame k when it
      is not empty (the whole frame when the depth changes sign at those corners).  A
      frame's areas are ordered by the partner camera.  FP64 throughout.
"""
from __future__ import annotations

import math

import numpy as np

SLACK = 1e-6


def footprint(H, w: int, h: int):
    """R37: (x0, y0, x1, y1) of the frame's corner images under H, or None when unbounded."""
    return _image_box(np.asarray(H, dtype=np.float64), 0.0, 0.0, float(w), float(h))


def _image_box(M, x0: float, y0: float, x1: float, y1: float):
    """Bounding box of the images of the rectangle's corners under the projective map M,
    or None when the depth changes sign or vanishes there."""
    pts = np.array([[x0, y0, 1.0], [x1, y0, 1.0], [x1, y1, 1.0], [x0, y1, 1.0]]) @ M.T
    z = pts[:, 2]
    if not (np.all(z > 0) or np.all(z < 0)):
        return None
    X, Y = pts[:, 0] / z, pts[:, 1] / z
    if not (np.all(np.isfinite(X)) and np.all(np.isfinite(Y))):
        return None
    return X.min(), Y.min(), X.max(), Y.max()


def detection_areas(frame_sizes, Hs, canvas_w: int, canvas_h: int, margin: int = 24):
    """Alg. 2 step 1 under R37: per camera, the list of areas (x, y, width, height)."""
    n = len(frame_sizes)
    F = [footprint(Hs[i], *frame_sizes[i]) for i in range(n)]
    out = [[] for _ in range(n)]
    for i in range(n):
        for j in range(i + 1, n):
            if F[i] is None or F[j] is None:
                continue
            ox0, oy0 = max(F[i][0], F[j][0]), max(F[i][1], F[j][1])
            ox1, oy1 = min(F[i][2], F[j][2]), min(F[i][3], F[j][3])
            if not (ox1 > ox0 and oy1 > oy0):
                continue
            ox0, oy0 = max(ox0 - margin, 0.0), max(oy0 - margin, 0.0)
            ox1, oy1 = min(ox1 + margin, float(canvas_w)), min(oy1 + margin, float(canvas_h))
            if not (ox1 > ox0 and oy1 > oy0):
                continue
            for k in (i, j):
                w, h = frame_sizes[k]
                box = _image_box(np.linalg.inv(np.asarray(Hs[k], dtype=np.float64)), ox0, oy0, ox1, oy1)
                if box is None:
                    x0, y0, x1, y1 = 0, 0, w, h
                else:
                    x0 = max(0, math.floor(box[0] - SLACK))
                    y0 = max(0, math.floor(box[1] - SLACK))
                    x1 = min(w, math.ceil(box[2] + SLACK))
                    y1 = min(h, math.ceil(box[3] + SLACK))
                if x1 > x0 and y1 > y0:
                    out[k].append((x0, y0, x1 - x0, y1 - y0))
    return out
