"""Plain CPU oracle of the L-ORB feature extraction (Sec. 4.1, Alg. 1 and Alg. 2).

TEST INFRASTRUCTURE ONLY: tests/ and bench.py may import it; the HIP product path never
does, and the two share no code, header, table or helper.

What is computed.  Within each feature detection area of a frame (Alg. 2, step 1), FAST
corners (Alg. 1, step 4) are scored with the Harris response R = det M - alpha (trace M)^2
of the Gaussian-weighted (sigma = 1) gradient products (Alg. 1, steps 1-3, 5), those with
R below a threshold t are dropped, non-maximal suppression keeps the local maxima
(Alg. 1, step 6) and the N of largest response remain (Alg. 1, step 7; Alg. 2, step 3).
Each kept point gets a BRIEF descriptor from n_d point pairs of the smoothed image
(Sec. 4.1.2; Alg. 2, step 4).  The paper fixes none of the operators or constants; the
readings (numbered after the stitching oracle's R1-R16) make every decision an exact
integer one, so a GPU implementation can match it bit for bit:

  R17 gray level g = (77 R + 150 G + 29 B + 128) >> 8 of the uint8 RGB frame.
  R18 FAST (Rosten's segment test, the 16-pixel circle of radius 3): p is a corner when
      at least 9 cyclically contiguous circle pixels c all have g(c) > g(p) + tf, or all
      have g(c) < g(p) - tf.
  R19 gradients by central differences: Ix = g(x+1, y) - g(x-1, y), Iy = g(x, y+1) -
      g(x, y-1) (integers, no factor 1/2).
  R20 Gaussian weighting with sigma = 1: the 5x5 binomial window b b^T, b = [1, 4, 6, 4, 1]
      (variance exactly 1 per axis), unnormalised: A = sum b b^T Ix^2, B = sum b b^T Iy^2,
      C = sum b b^T Ix Iy (integers).
  R21 alpha = 3/64 (inside the customary 0.04 - 0.06) and the response scaled by 64, so it
      is an integer: R = 64 (A B - C^2) - 3 (A + B)^2.
  R22 a candidate is a FAST corner of the area with R >= t (Alg. 1, step 5 deletes the
      points whose response is less than t).
  R23 non-maximal suppression over the 3x3 neighbourhood among candidates: p survives
      when every neighbouring candidate q has R(q) < R(p), or R(q) = R(p) and q comes
      later in raster order (index y * w + x).
  R24 the N survivors of largest R, ties by raster index, in that order.
  R25 BRIEF on the smoothed image S = b b^T * g (the same binomial window, integer sums):
      for each pair k of offsets (p_k, q_k) inside the 31x31 patch (|dx|, |dy| <= 15) the
      paper's three-valued test gives +1 when S(x + p_k) > S(x + q_k), -1 when <, 0 when
      equal; it is kept as two bit strings (gt, lt).  The pairs are an input (a seeded
      pattern), not a property of the method.
  R26 only points whose descriptor support lies in the frame are considered: 17 <= x < w
      - 17 and 17 <= y < h - 17 (15 for the patch, 2 for the smoothing window); the
      detection areas are rectangles in frame coordinates, clipped to that range.
"""
from __future__ import annotations

import numpy as np

B5 = np.array([1, 4, 6, 4, 1], dtype=np.int64)
# the FAST circle of radius 3, clockwise from the top
CIRCLE = [(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
          (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)]
MARGIN = 17
ALPHA_NUM, ALPHA_DEN = 3, 64


def gray(rgb: np.ndarray) -> np.ndarray:
    """R17: integer luma of an (h, w, 3) uint8 frame."""
    c = rgb.astype(np.int64)
    return (77 * c[..., 0] + 150 * c[..., 1] + 29 * c[..., 2] + 128) >> 8


def fast_corner(g: np.ndarray, x: int, y: int, tf: int) -> bool:
    """R18: the segment test at (x, y); the circle must lie in the image."""
    p = int(g[y, x])
    ring = [int(g[y + dy, x + dx]) for dx, dy in CIRCLE]
    for sign in (1, -1):
        hit = [(sign * (v - p)) > tf for v in ring]
        run = 0
        for k in range(32):              # twice round the circle: runs that wrap
            run = run + 1 if hit[k % 16] else 0
            if run >= 9:
                return True
    return False


def structure(g: np.ndarray, x: int, y: int):
    """R19-R20: A, B, C of the binomially weighted gradient products at (x, y)."""
    A = B = C = 0
    for j in range(-2, 3):
        for i in range(-2, 3):
            w = int(B5[j + 2] * B5[i + 2])
            u, v = x + i, y + j
            ix = int(g[v, u + 1]) - int(g[v, u - 1])
            iy = int(g[v + 1, u]) - int(g[v - 1, u])
            A += w * ix * ix
            B += w * iy * iy
            C += w * ix * iy
    return A, B, C


def harris(g: np.ndarray, x: int, y: int) -> int:
    """R21: 64 det M - 3 (trace M)^2."""
    A, B, C = structure(g, x, y)
    return ALPHA_DEN * (A * B - C * C) - ALPHA_NUM * (A + B) ** 2


def smooth(g: np.ndarray) -> np.ndarray:
    """R25: S = b b^T * g on the interior (2 samples from each edge); int64, zeros at the
    border rows and columns (never read under R26)."""
    h, w = g.shape
    S = np.zeros((h, w), dtype=np.int64)
    for j in range(-2, 3):
        for i in range(-2, 3):
            S[2:h - 2, 2:w - 2] += B5[j + 2] * B5[i + 2] * g[2 + j:h - 2 + j, 2 + i:w - 2 + i]
    return S


def clip_area(rect, w: int, h: int):
    """R26: the area (x, y, width, height) clipped to the descriptor-support range."""
    x0, y0, rw, rh = rect
    x1, y1 = min(x0 + rw, w - MARGIN), min(y0 + rh, h - MARGIN)
    x0, y0 = max(x0, MARGIN), max(y0, MARGIN)
    return x0, y0, max(0, x1 - x0), max(0, y1 - y0)


def candidates(g: np.ndarray, rect, tf: int, t: int) -> dict:
    """R22: {(x, y): R} for the FAST corners of the clipped area with R >= t."""
    h, w = g.shape
    x0, y0, rw, rh = clip_area(rect, w, h)
    out = {}
    for y in range(y0, y0 + rh):
        for x in range(x0, x0 + rw):
            if fast_corner(g, x, y, tf):
                r = harris(g, x, y)
                if r >= t:
                    out[(x, y)] = r
    return out


def suppress(cand: dict, w: int) -> list:
    """R23: the candidates that are maxima of their 3x3 neighbourhood (ties to the first
    in raster order)."""
    keep = []
    for (x, y), r in cand.items():
        idx = y * w + x
        ok = True
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dx or dy) and (x + dx, y + dy) in cand:
                    rq = cand[(x + dx, y + dy)]
                    iq = (y + dy) * w + (x + dx)
                    if not (rq < r or (rq == r and iq > idx)):
                        ok = False
        if ok:
            keep.append((x, y, r))
    return keep


def select(keep: list, n: int, w: int) -> list:
    """R24: the n survivors of largest R, ties by raster index."""
    return sorted(keep, key=lambda k: (-k[2], k[1] * w + k[0]))[:n]


def brief(S: np.ndarray, x: int, y: int, pattern: np.ndarray):
    """R25: (gt, lt) bit arrays of the pattern's pairs (rows dx1, dy1, dx2, dy2)."""
    a = S[y + pattern[:, 1], x + pattern[:, 0]]
    b = S[y + pattern[:, 3], x + pattern[:, 2]]
    return (a > b), (a < b)


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """Bit k of the string -> bit (k % 32) of 32-bit word k // 32."""
    bits = np.asarray(bits, dtype=np.uint64).reshape(-1, 32)
    return (bits << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)


def lorb(rgb: np.ndarray, areas, tf: int, t: int, n: int, pattern: np.ndarray):
    """Alg. 2 on one frame: per area, the selected points [(x, y, R)] and their descriptors
    as packed words (gt words, then lt words)."""
    g = gray(rgb)
    h, w = g.shape
    S = smooth(g)
    out = []
    for rect in areas:
        pts = select(suppress(candidates(g, rect, tf, t), w), n, w)
        desc = []
        for x, y, _ in pts:
            gt, lt = brief(S, x, y, pattern)
            desc.append(np.concatenate([pack_bits(gt), pack_bits(lt)]))
        words = 2 * ((len(pattern) + 31) // 32)
        out.append((pts, np.array(desc, dtype=np.uint32).reshape(len(pts), words)))
    return out
