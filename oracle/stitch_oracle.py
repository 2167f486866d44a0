"""Plain FP64 CPU oracle of the per-frame panorama stitching path.

TEST INFRASTRUCTURE ONLY: tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import it; the HIP product path never does.  It shares no
code, header, table or helper with the HIP path.

What is computed.  The paper's stitcher transforms each camera's video with fixed,
pre-corrected parameters (Alg. 4, step 1), then transforms the video and blends it
into the panorama (Alg. 4, step 6), removing seams with "multi band fusion"
(Sec. 1, contribution 3).  The paper gives no interpolation rule, filter, border
rule or level count; this oracle follows the textbook multi-band method
(Burt & Adelson's Laplacian-pyramid multiresolution spline, generating kernel
a = 0.375) under these readings:

  R1  pixel (x, y) = (column, row) is a sample at integer coordinates.
  R2  H maps source -> canvas; the warp pulls through H^-1.
  R3  H^-1 := adj(H) / adj(H)[2,2] in FP64 (cofactors as a*b - c*d), each entry
      rounded to FP32; canvas coordinates X, Y become FP32; u, v, z are evaluated as
      (h0*X + h1*Y) + h2 with FP32 round-to-nearest at every operation and no fused
      multiply-add; a sample with !(z > 0) is 0; x = u/z, y = v/z in FP32;
      x0 = floor(x), fx = x - x0 (exact).  Everything after that is FP64.
  R4  bilinear interpolation of p = u8/255; a tap outside the frame contributes 0.
  R5  borders: reflect-101 (index -i -> i, (n-1)+i -> (n-1)-i); every level side >= 3.
  R6  REDUCE: G'[y,x] = sum_{a,b} w_a w_b G[f(2y+a-2), f(2x+b-2)], w = [1,4,6,4,1]/16,
      level sides ceil(n/2).
  R7  EXPAND to a fine size n: E[y,x] = 4 sum_{a,b} w_a w_b u[f(y+a-2), f(x+b-2)],
      u = coarse samples placed at even fine indices, zeros at odd ones, folded in
      the fine domain.
  R8  L_k = G_k - EXPAND(G_{k+1}) for k < L-1, L_{L-1} = G_{L-1}; "L levels" = L arrays.
  R9  masks: uint8 weights per camera on the canvas, summing to 255 at every pixel;
      m = u8/255; mask pyramid = REDUCE chain of m.
  R11 B_k = sum_i Gm_i^k * L_i^k; R_{L-1} = B_{L-1}; R_k = B_k + EXPAND(R_{k+1});
      output = clip(rint(255 R_0), 0, 255) as uint8 (round half to even).
  R12 every per-camera array lives on the whole canvas (zero outside the frame's
      footprint, reflect-101 at canvas edges).

"coords='ideal'" replaces R3 by the exact FP64 inverse, for fidelity reports.
Arrays are channel-first (C, rows, cols) float64; frames are (h, w, 3) uint8.
"""
from __future__ import annotations

import numpy as np

W5 = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


# ----------------------------------------------------------------------------- geometry
def level_dims(h: int, w: int, levels: int) -> list[tuple[int, int]]:
    """Level-k sides: d_k = ceil(d_{k-1} / 2) (R6)."""
    dims = [(int(h), int(w))]
    for _ in range(levels - 1):
        ph, pw = dims[-1]
        dims.append(((ph + 1) // 2, (pw + 1) // 2))
    return dims


def reflect101(i, n: int) -> np.ndarray:
    """Reflect-101 fold of integer indices into [0, n) (R5); overshoot must be < n."""
    if n < 3:
        raise ValueError(f"level side {n} < 3: reflect-101 with a 5-tap kernel is undefined")
    i = np.asarray(i, dtype=np.int64)
    j = np.where(i < 0, -i, i)
    j = np.where(j > n - 1, 2 * (n - 1) - j, j)
    if np.any((j < 0) | (j > n - 1)):
        raise ValueError("index overshoots the side by more than one reflection")
    return j


def _adjugate(H: np.ndarray) -> np.ndarray:
    """adj(H) with each cofactor formed as a*b - c*d in FP64 (R3)."""
    a = np.asarray(H, dtype=np.float64).reshape(3, 3)
    adj = np.empty((3, 3))
    adj[0, 0] = a[1, 1] * a[2, 2] - a[1, 2] * a[2, 1]
    adj[0, 1] = a[0, 2] * a[2, 1] - a[0, 1] * a[2, 2]
    adj[0, 2] = a[0, 1] * a[1, 2] - a[0, 2] * a[1, 1]
    adj[1, 0] = a[1, 2] * a[2, 0] - a[1, 0] * a[2, 2]
    adj[1, 1] = a[0, 0] * a[2, 2] - a[0, 2] * a[2, 0]
    adj[1, 2] = a[0, 2] * a[1, 0] - a[0, 0] * a[1, 2]
    adj[2, 0] = a[1, 0] * a[2, 1] - a[1, 1] * a[2, 0]
    adj[2, 1] = a[0, 1] * a[2, 0] - a[0, 0] * a[2, 1]
    adj[2, 2] = a[0, 0] * a[1, 1] - a[0, 1] * a[1, 0]
    return adj


def hinv_ideal(H) -> np.ndarray:
    """FP64 canvas -> source map adj(H)/adj(H)[2,2] (R2, R3 step 1 before rounding)."""
    a = np.asarray(H, dtype=np.float64).reshape(3, 3)
    if not np.all(np.isfinite(a)):
        raise ValueError("homography has a non-finite entry")
    adj = _adjugate(a)
    if adj[2, 2] == 0.0 or not np.all(np.isfinite(adj)):
        raise ValueError("homography inverse cannot be normalised (adj[2,2] == 0)")
    out = adj / adj[2, 2]
    if not np.all(np.isfinite(out)):
        raise ValueError("normalised inverse is not finite")
    return out


def hinv_spec(H) -> np.ndarray:
    """R3 step 1: the FP64 normalised adjugate rounded entrywise to FP32."""
    out = hinv_ideal(H).astype(np.float32)
    if not np.all(np.isfinite(out)):
        raise ValueError("normalised inverse overflows FP32")
    return out


# ----------------------------------------------------------------------------- warp
def warp_coords(hinv: np.ndarray, rows, cols):
    """Source coordinates (x, y) of the canvas grid rows x cols and the in-range flag (R3).

    hinv float32: the FP32 sequence of R3 (numpy applies one IEEE round-to-nearest per
    ufunc, so no operation is fused).  hinv float64: FP64 coordinates.  The third
    result is the flag z > 0; whether any tap falls inside the frame is the caller's test."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    ft = np.float32 if hinv.dtype == np.float32 else np.float64
    g = hinv.ravel().astype(ft)
    X = cols.astype(ft)[None, :]
    Y = rows.astype(ft)[:, None]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        u = (g[0] * X + g[1] * Y) + g[2]
        v = (g[3] * X + g[4] * Y) + g[5]
        z = (g[6] * X + g[7] * Y) + g[8]
        x = u / z
        y = v / z
    return x, y, z > 0


def warp(src: np.ndarray, hinv: np.ndarray, rows, cols) -> np.ndarray:
    """G_0 on the canvas grid rows x cols (R1-R4).  hinv float32 -> R3 coordinate
    sequence; hinv float64 -> exact FP64 coordinates.  Returns (3, R, C) float64."""
    src = np.asarray(src)
    h, w = src.shape[:2]
    ft = np.float32 if hinv.dtype == np.float32 else np.float64
    x, y, zpos = warp_coords(hinv, rows, cols)
    with np.errstate(invalid="ignore"):
        ok = zpos & (x >= -1) & (x < w) & (y >= -1) & (y < h)
        x = np.where(ok, x, ft(0))
        y = np.where(ok, y, ft(0))
        x0 = np.floor(x)
        y0 = np.floor(y)
        fx = (x - x0).astype(np.float64)
        fy = (y - y0).astype(np.float64)
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)

    def tap(dy, dx):
        yy = y0 + dy
        xx = x0 + dx
        inside = ok & (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
        vals = src[np.clip(yy, 0, h - 1), np.clip(xx, 0, w - 1), :].astype(np.float64) / 255.0
        return np.where(inside[..., None], vals, 0.0)

    p00, p01, p10, p11 = tap(0, 0), tap(0, 1), tap(1, 0), tap(1, 1)
    fx = fx[..., None]
    fy = fy[..., None]
    val = (1.0 - fy) * ((1.0 - fx) * p00 + fx * p01) + fy * ((1.0 - fx) * p10 + fx * p11)
    val = np.where(ok[..., None], val, 0.0)
    return np.moveaxis(val, -1, 0)


# ----------------------------------------------------------------------------- filters
def reduce_at(fetch, n_y: int, n_x: int, rows, cols) -> np.ndarray:
    """R6 at coarse indices rows x cols; fetch(R, C) returns the finer level (n_y x n_x)
    on the index grid R x C as (..., len(R), len(C))."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    ty = [reflect101(2 * rows + a - 2, n_y) for a in range(5)]
    tx = [reflect101(2 * cols + b - 2, n_x) for b in range(5)]
    RR = np.unique(np.concatenate(ty))
    CC = np.unique(np.concatenate(tx))
    g = fetch(RR, CC)
    out = np.zeros(g.shape[:-2] + (len(rows), len(cols)))
    for a in range(5):
        ia = np.searchsorted(RR, ty[a])
        for b in range(5):
            ib = np.searchsorted(CC, tx[b])
            out += (W5[a] * W5[b]) * g[..., ia[:, None], ib[None, :]]
    return out


def expand_at(fetch_coarse, n_y: int, n_x: int, rows, cols) -> np.ndarray:
    """R7 at fine indices rows x cols of a fine level of size n_y x n_x; fetch_coarse(R, C)
    returns the coarse level on the index grid R x C."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    ty = [reflect101(rows + a - 2, n_y) for a in range(5)]
    tx = [reflect101(cols + b - 2, n_x) for b in range(5)]
    ey = [t % 2 == 0 for t in ty]
    ex = [t % 2 == 0 for t in tx]
    RR = np.unique(np.concatenate([t[e] // 2 for t, e in zip(ty, ey)]))
    CC = np.unique(np.concatenate([t[e] // 2 for t, e in zip(tx, ex)]))
    g = fetch_coarse(RR, CC)
    out = np.zeros(g.shape[:-2] + (len(rows), len(cols)))
    for a in range(5):
        ia = np.minimum(np.searchsorted(RR, ty[a] // 2), len(RR) - 1)
        for b in range(5):
            ib = np.minimum(np.searchsorted(CC, tx[b] // 2), len(CC) - 1)
            even = ey[a][:, None] & ex[b][None, :]
            out += (4.0 * W5[a] * W5[b]) * np.where(even, g[..., ia[:, None], ib[None, :]], 0.0)
    return out


def _grid_fetch(arr):
    return lambda R, C: arr[..., R[:, None], C[None, :]]


def reduce_full(g: np.ndarray) -> np.ndarray:
    """REDUCE of a whole array (..., n_y, n_x) -> (..., ceil(n_y/2), ceil(n_x/2))."""
    n_y, n_x = g.shape[-2:]
    return reduce_at(_grid_fetch(np.asarray(g, dtype=np.float64)), n_y, n_x,
                     np.arange((n_y + 1) // 2), np.arange((n_x + 1) // 2))


def expand_full(g: np.ndarray, n_y: int, n_x: int) -> np.ndarray:
    """EXPAND of a whole coarse array to the fine size n_y x n_x."""
    return expand_at(_grid_fetch(np.asarray(g, dtype=np.float64)), n_y, n_x,
                     np.arange(n_y), np.arange(n_x))


def gaussian_pyramid(img: np.ndarray, levels: int) -> list[np.ndarray]:
    """[G_0 .. G_{L-1}] with G_{k+1} = REDUCE(G_k) (R6)."""
    out = [np.asarray(img, dtype=np.float64)]
    for _ in range(levels - 1):
        out.append(reduce_full(out[-1]))
    return out


def laplacian_pyramid(img: np.ndarray, levels: int) -> list[np.ndarray]:
    """[L_0 .. L_{L-1}] (R8)."""
    g = gaussian_pyramid(img, levels)
    out = []
    for k in range(levels - 1):
        n_y, n_x = g[k].shape[-2:]
        out.append(g[k] - expand_full(g[k + 1], n_y, n_x))
    out.append(g[-1])
    return out


def collapse(lap: list[np.ndarray]) -> np.ndarray:
    """R_{L-1} = L_{L-1}; R_k = L_k + EXPAND(R_{k+1}); returns R_0."""
    r = lap[-1]
    for k in range(len(lap) - 2, -1, -1):
        n_y, n_x = lap[k].shape[-2:]
        r = lap[k] + expand_full(r, n_y, n_x)
    return r


def blend_pyramids(laps: list[list[np.ndarray]], gms: list[list[np.ndarray]]) -> list[np.ndarray]:
    """R11: per-level mask-weighted sums B_k, collapsed; returns [R_0 .. R_{L-1}]."""
    levels = len(laps[0])
    bands = []
    for k in range(levels):
        acc = np.zeros_like(laps[0][k])
        for lap, gm in zip(laps, gms):
            acc = acc + gm[k] * lap[k]
        bands.append(acc)
    rs = [None] * levels
    rs[-1] = bands[-1]
    for k in range(levels - 2, -1, -1):
        n_y, n_x = bands[k].shape[-2:]
        rs[k] = bands[k] + expand_full(rs[k + 1], n_y, n_x)
    return rs


def quantise(r0: np.ndarray) -> np.ndarray:
    """R11 output: (3, H, W) float -> (H, W, 3) uint8 via clip(rint(255 r), 0, 255)."""
    q = np.clip(np.rint(255.0 * np.asarray(r0, dtype=np.float64)), 0.0, 255.0)
    return np.moveaxis(q, 0, -1).astype(np.uint8)


def check_masks(masks, canvas_w: int, canvas_h: int) -> None:
    """R9: one uint8 weight map per camera on the canvas, summing to 255 everywhere."""
    total = np.zeros((canvas_h, canvas_w), dtype=np.int64)
    for m in masks:
        m = np.asarray(m)
        if m.shape != (canvas_h, canvas_w) or m.dtype != np.uint8:
            raise ValueError("each mask must be a (canvas_h, canvas_w) uint8 array")
        total += m
    if np.any(total != 255):
        raise ValueError("mask weights must sum to 255 at every canvas pixel")


# ----------------------------------------------------------------------------- whole path
class StitchOracle:
    """The whole path of R1-R12 for one frame set, evaluable on any canvas index grid.

    Every quantity X(level, rows, cols) is computed from its definition on exactly the
    indices it needs, so a small window of a huge canvas costs only its dependency
    cone, and the full canvas is the case rows = arange(H_k), cols = arange(W_k).
    Results are memoised per (quantity, index grid)."""

    def __init__(self, frames, Hs, masks, canvas_w: int, canvas_h: int, levels: int,
                 coords: str = "spec"):
        if len(frames) != len(Hs) or len(frames) != len(masks) or len(frames) < 1:
            raise ValueError("need one frame, one homography and one mask per camera")
        self.frames = [np.asarray(f, dtype=np.uint8) for f in frames]
        for f in self.frames:
            if f.ndim != 3 or f.shape[2] != 3:
                raise ValueError("frames are (h, w, 3) uint8")
        self.masks = [np.asarray(m, dtype=np.uint8) for m in masks]
        check_masks(self.masks, canvas_w, canvas_h)
        self.levels = int(levels)
        if self.levels < 1:
            raise ValueError("levels must be >= 1")
        self.dims = level_dims(canvas_h, canvas_w, self.levels)
        if min(min(d) for d in self.dims) < 3:
            raise ValueError("every level side must be >= 3")
        if coords == "spec":
            self.hinv = [hinv_spec(H) for H in Hs]
        elif coords == "ideal":
            self.hinv = [hinv_ideal(H) for H in Hs]
        else:
            raise ValueError("coords is 'spec' or 'ideal'")
        self.n = len(self.frames)
        self._memo = {}

    def clear(self) -> None:
        self._memo.clear()

    def _grid(self, k, rows, cols):
        H, W = self.dims[k]
        rows = np.arange(H, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
        cols = np.arange(W, dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
        if rows.size and (rows.min() < 0 or rows.max() >= H):
            raise IndexError("row outside the level")
        if cols.size and (cols.min() < 0 or cols.max() >= W):
            raise IndexError("column outside the level")
        return rows, cols

    def _memoised(self, key, rows, cols, fn):
        mk = key + (rows.tobytes(), cols.tobytes())
        hit = self._memo.get(mk)
        if hit is None:
            hit = fn(rows, cols)
            self._memo[mk] = hit
        return hit

    def G(self, i, k, rows=None, cols=None):
        """Gaussian level k of camera i's warped frame (3, R, C)."""
        rows, cols = self._grid(k, rows, cols)
        if k == 0:
            return self._memoised(("G", i, 0), rows, cols,
                                  lambda r, c: warp(self.frames[i], self.hinv[i], r, c))
        n_y, n_x = self.dims[k - 1]
        return self._memoised(("G", i, k), rows, cols, lambda r, c: reduce_at(
            lambda R, C: self.G(i, k - 1, R, C), n_y, n_x, r, c))

    def Gm(self, i, k, rows=None, cols=None):
        """Gaussian level k of camera i's mask (1, R, C)."""
        rows, cols = self._grid(k, rows, cols)
        if k == 0:
            return self._memoised(("Gm", i, 0), rows, cols, lambda r, c: (
                self.masks[i][r[:, None], c[None, :]].astype(np.float64) / 255.0)[None])
        n_y, n_x = self.dims[k - 1]
        return self._memoised(("Gm", i, k), rows, cols, lambda r, c: reduce_at(
            lambda R, C: self.Gm(i, k - 1, R, C), n_y, n_x, r, c))

    def Lap(self, i, k, rows=None, cols=None):
        """Laplacian level k of camera i (R8)."""
        rows, cols = self._grid(k, rows, cols)
        if k == self.levels - 1:
            return self.G(i, k, rows, cols)
        n_y, n_x = self.dims[k]
        return self._memoised(("L", i, k), rows, cols, lambda r, c: self.G(i, k, r, c) - expand_at(
            lambda R, C: self.G(i, k + 1, R, C), n_y, n_x, r, c))

    def B(self, k, rows=None, cols=None):
        """Blended band k (R11)."""
        rows, cols = self._grid(k, rows, cols)

        def fn(r, c):
            acc = np.zeros((3, len(r), len(c)))
            for i in range(self.n):
                acc = acc + self.Gm(i, k, r, c) * self.Lap(i, k, r, c)
            return acc
        return self._memoised(("B", k), rows, cols, fn)

    def R(self, k, rows=None, cols=None):
        """Collapsed level k (R11)."""
        rows, cols = self._grid(k, rows, cols)
        if k == self.levels - 1:
            return self.B(k, rows, cols)
        n_y, n_x = self.dims[k]
        return self._memoised(("R", k), rows, cols, lambda r, c: self.B(k, r, c) + expand_at(
            lambda R_, C_: self.R(k + 1, R_, C_), n_y, n_x, r, c))

    def panorama(self, rows=None, cols=None) -> np.ndarray:
        """uint8 (R, C, 3) panorama on the requested canvas grid."""
        return quantise(self.R(0, rows, cols))
