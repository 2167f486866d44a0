"""FP64 oracle of the stitching path's adjoint (TEST INFRASTRUCTURE ONLY, like the
rest of oracle/): the gradient of an overlap photometric loss after warp + multi-band
blend with respect to the source pixels and the 8 corner parameters of a homography.

The paper registers frames by feature matching and PROSAC (Alg. 3, Alg. 4 step 5) and
then stitches with the fixed transformation (Alg. 4 steps 1 and 6); it has no gradient.
This differentiable form refines that transformation by gradient descent on the same
stitched output, under these readings:

  * frames are float images in [0, 1] (channel-first), so a pixel gradient exists;
  * camera 0 has a fixed map, camera 1's source -> canvas homography H(q) is the
    direct linear transform of its four corners (0,0), (w-1,0), (w-1,h-1), (0,h-1)
    to the canvas points q (8 numbers, h33 = 1);
  * loss  l = 1/(6|Omega|) * sum_{p in Omega, c} (P_c - A_c)^2 + (P_c - B_c)^2, with P the
    blended R_0 (float, before quantisation), A and B the warped frames G_0, and Omega
    the canvas pixels where both frames have all four bilinear taps inside and z > 0;
  * for differentiation the bilinear cells (x0, y0) and Omega are frozen at a reference
    map, so l is smooth in q; at integers the cell is [x0, x0+1] (right derivative);
  * warp, pyramids and blend follow the forward oracle's definitions (stitch_oracle).

Transposes are written from the forward definitions: every tap of REDUCE / EXPAND /
bilinear interpolation is scattered back with np.add.at.
"""
from __future__ import annotations

import numpy as np

from .stitch_oracle import W5, hinv_ideal, level_dims, reflect101, reduce_full, expand_full


# ----------------------------------------------------------------------------- homography
def corners(w: int, h: int) -> np.ndarray:
    return np.array([[0.0, 0.0], [w - 1.0, 0.0], [w - 1.0, h - 1.0], [0.0, h - 1.0]])


def dlt_from_corners(q, w: int, h: int) -> np.ndarray:
    """H (h33 = 1) mapping the frame corners to the canvas points q (x0,y0,...,x3,y3)."""
    q = np.asarray(q, dtype=np.float64).reshape(4, 2)
    A = np.zeros((8, 8))
    b = np.zeros(8)
    for k, ((x, y), (X, Y)) in enumerate(zip(corners(w, h), q)):
        A[2 * k] = [x, y, 1.0, 0.0, 0.0, 0.0, -X * x, -X * y]
        A[2 * k + 1] = [0.0, 0.0, 0.0, x, y, 1.0, -Y * x, -Y * y]
        b[2 * k], b[2 * k + 1] = X, Y
    hv = np.linalg.solve(A, b)
    return np.append(hv, 1.0).reshape(3, 3)


def dlt_jacobian(q, w: int, h: int) -> np.ndarray:
    """d vec(H) / d q (9 x 8), from differentiating A(q) h = b(q)."""
    q = np.asarray(q, dtype=np.float64).reshape(4, 2)
    A = np.zeros((8, 8))
    b = np.zeros(8)
    for k, ((x, y), (X, Y)) in enumerate(zip(corners(w, h), q)):
        A[2 * k] = [x, y, 1.0, 0.0, 0.0, 0.0, -X * x, -X * y]
        A[2 * k + 1] = [0.0, 0.0, 0.0, x, y, 1.0, -Y * x, -Y * y]
        b[2 * k], b[2 * k + 1] = X, Y
    hv = np.linalg.solve(A, b)
    J = np.zeros((9, 8))
    for k, (x, y) in enumerate(corners(w, h)):
        for d in range(2):                       # d = 0: X_k, d = 1: Y_k
            dA = np.zeros((8, 8))
            db = np.zeros(8)
            row = 2 * k + d
            dA[row, 6], dA[row, 7] = -x, -y
            db[row] = 1.0
            J[:8, 2 * k + d] = np.linalg.solve(A, db - dA @ hv)
    return J


def canvas_map_jacobian(H: np.ndarray) -> np.ndarray:
    """d vec(M) / d vec(H) (9 x 9) for M = N / N[2,2], N = H^-1 (the warp's pull map)."""
    N = np.linalg.inv(H)
    n22 = N[2, 2]
    J = np.zeros((9, 9))
    for j in range(9):
        dH = np.zeros((3, 3))
        dH.flat[j] = 1.0
        dN = -N @ dH @ N
        dM = dN / n22 - N * dN[2, 2] / n22 ** 2
        J[:, j] = dM.ravel()
    return J


# ----------------------------------------------------------------------------- transposes
def reduce_T(d: np.ndarray, n_y: int, n_x: int) -> np.ndarray:
    """Transpose of REDUCE: scatter every tap of the coarse gradient to the fine level."""
    out = np.zeros(d.shape[:-2] + (n_y, n_x))
    m_y, m_x = d.shape[-2:]
    ys, xs = np.arange(m_y), np.arange(m_x)
    for a in range(5):
        ty = reflect101(2 * ys + a - 2, n_y)
        for b in range(5):
            tx = reflect101(2 * xs + b - 2, n_x)
            np.add.at(out, (..., ty[:, None], tx[None, :]), (W5[a] * W5[b]) * d)
    return out


def expand_T(d: np.ndarray) -> np.ndarray:
    """Transpose of EXPAND to the fine size of d: scatter to the zero-inserted signal,
    keep its even samples."""
    n_y, n_x = d.shape[-2:]
    u = np.zeros(d.shape)
    ys, xs = np.arange(n_y), np.arange(n_x)
    for a in range(5):
        ty = reflect101(ys + a - 2, n_y)
        for b in range(5):
            tx = reflect101(xs + b - 2, n_x)
            np.add.at(u, (..., ty[:, None], tx[None, :]), (4.0 * W5[a] * W5[b]) * d)
    return u[..., ::2, ::2]


# ----------------------------------------------------------------------------- differentiable path
class GradOracle:
    """Loss and analytic gradients for float frames, with frozen cells and Omega.

    frames: list of (3, h, w) float64 in [0, 1]; masks: uint8 canvas weights (sum 255);
    coords: 'spec' (FP32 coordinate sequence of the forward path) or 'ideal' (FP64)."""

    def __init__(self, frames, masks, canvas_w: int, canvas_h: int, levels: int, coords: str = "ideal"):
        self.frames = [np.asarray(f, dtype=np.float64) for f in frames]
        if len(self.frames) != 2:
            raise ValueError("the overlap loss is defined on a pair of frames")
        self.masks = [np.asarray(m, dtype=np.uint8) for m in masks]
        self.W, self.H, self.L = canvas_w, canvas_h, levels
        self.dims = level_dims(canvas_h, canvas_w, levels)
        self.coords = coords
        self.gm = [self._gauss(m[None].astype(np.float64) / 255.0) for m in self.masks]

    def _gauss(self, img):
        out = [img]
        for _ in range(self.L - 1):
            out.append(reduce_full(out[-1]))
        return out

    def _map(self, H):
        M = hinv_ideal(H)
        return M.astype(np.float32) if self.coords == "spec" else M

    def _coords(self, M):
        ft = np.float32 if M.dtype == np.float32 else np.float64
        g = M.ravel().astype(ft)
        X = np.arange(self.W, dtype=ft)[None, :]
        Y = np.arange(self.H, dtype=ft)[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = (g[0] * X + g[1] * Y) + g[2]
            v = (g[3] * X + g[4] * Y) + g[5]
            z = (g[6] * X + g[7] * Y) + g[8]
            x = (u / z).astype(np.float64)
            y = (v / z).astype(np.float64)
        return x, y, z.astype(np.float64) > 0

    def cells(self, Hs):
        """Frozen cells (x0, y0) of both cameras and Omega at the maps Hs."""
        out, omega = [], np.ones((self.H, self.W), bool)
        for f, H in zip(self.frames, Hs):
            h, w = f.shape[1:]
            x, y, zpos = self._coords(self._map(H))
            with np.errstate(invalid="ignore"):
                x0 = np.where(zpos & np.isfinite(x), np.floor(x), -10).astype(np.int64)
                y0 = np.where(zpos & np.isfinite(y), np.floor(y), -10).astype(np.int64)
            omega &= zpos & (x0 >= 0) & (x0 + 1 <= w - 1) & (y0 >= 0) & (y0 + 1 <= h - 1)
            out.append((x0, y0))
        return out, omega

    def _warp(self, f, M, cell):
        """Bilinear of the float frame through M with the frozen cell; taps outside are 0."""
        h, w = f.shape[1:]
        x, y, zpos = self._coords(M)
        x0, y0 = cell
        fx = np.where(zpos, x - x0, 0.0)
        fy = np.where(zpos, y - y0, 0.0)

        def tap(dy, dx):
            yy, xx = y0 + dy, x0 + dx
            ok = zpos & (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
            return np.where(ok[None], f[:, np.clip(yy, 0, h - 1), np.clip(xx, 0, w - 1)], 0.0), ok

        (p00, k00), (p01, k01), (p10, k10), (p11, k11) = tap(0, 0), tap(0, 1), tap(1, 0), tap(1, 1)
        val = (1 - fy) * ((1 - fx) * p00 + fx * p01) + fy * ((1 - fx) * p10 + fx * p11)
        return val, dict(x=x, y=y, x0=x0, y0=y0, fx=fx, fy=fy, zpos=zpos, p=(p00, p01, p10, p11),
                         ok=(k00, k01, k10, k11))

    def forward(self, Hs, frozen):
        cells, omega = frozen
        Ms = [self._map(H) for H in Hs]
        Gs, aux = [], []
        for f, M, cell in zip(self.frames, Ms, cells):
            g, a = self._warp(f, M, cell)
            Gs.append(g)
            aux.append(a)
        laps = []
        for g in Gs:
            gp = [g]
            for _ in range(self.L - 1):
                gp.append(reduce_full(gp[-1]))
            lp = [gp[k] - expand_full(gp[k + 1], *gp[k].shape[-2:]) for k in range(self.L - 1)] + [gp[-1]]
            laps.append(lp)
        B = [sum(self.gm[i][k] * laps[i][k] for i in range(2)) for k in range(self.L)]
        R = B[-1]
        for k in range(self.L - 2, -1, -1):
            R = B[k] + expand_full(R, *B[k].shape[-2:])
        P = R
        n = omega.sum()
        loss = float(np.sum(((P - Gs[0]) ** 2 + (P - Gs[1]) ** 2)[:, omega]) / (6.0 * n))
        return dict(loss=loss, P=P, G=Gs, aux=aux, M=Ms, omega=omega, n=n)

    def loss(self, Hs, frozen) -> float:
        return self.forward(Hs, frozen)["loss"]

    def backward(self, st):
        """d loss / d frames (per camera) and d loss / d M (per camera, 3x3)."""
        P, G, omega, n = st["P"], st["G"], st["omega"], st["n"]
        om = omega[None].astype(np.float64)
        gP = (2.0 / (6.0 * n)) * ((P - G[0]) + (P - G[1])) * om
        gdir = [-(2.0 / (6.0 * n)) * (P - G[i]) * om for i in range(2)]
        L = self.L
        dB = [gP]
        for k in range(L - 1):
            dB.append(expand_T(dB[-1]))
        d_frames, d_M = [], []
        for i in range(2):
            dLk = [self.gm[i][k] * dB[k] for k in range(L)]
            if L == 1:
                dG0 = dLk[0]
            else:
                dG = dLk[L - 1] - expand_T(dLk[L - 2])
                for k in range(L - 2, 0, -1):
                    dG = dLk[k] - expand_T(dLk[k - 1]) + reduce_T(dG, *self.dims[k])
                dG0 = dLk[0] + reduce_T(dG, *self.dims[0])
            dG0 = dG0 + gdir[i]
            df, dm = self._warp_T(i, dG0, st["aux"][i], st["M"][i])
            d_frames.append(df)
            d_M.append(dm)
        return d_frames, d_M

    def _warp_T(self, i, dG, a, M):
        f = self.frames[i]
        h, w = f.shape[1:]
        x0, y0 = a["x0"], a["y0"]            # the frozen cell
        fx, fy = a["fx"], a["fy"]
        wts = [(1 - fy) * (1 - fx), (1 - fy) * fx, fy * (1 - fx), fy * fx]
        offs = [(0, 0), (0, 1), (1, 0), (1, 1)]
        df = np.zeros_like(f)
        for wt, (dy, dx), ok in zip(wts, offs, a["ok"]):
            yy, xx = y0 + dy, x0 + dx
            sel = ok
            for c in range(3):
                np.add.at(df[c], (yy[sel], xx[sel]), (wt * dG[c])[sel])
        p00, p01, p10, p11 = a["p"]
        dval_dx = (1 - fy) * (p01 - p00) + fy * (p11 - p10)
        dval_dy = (1 - fx) * (p10 - p00) + fx * (p11 - p01)
        gx = np.sum(dG * dval_dx, axis=0) * a["zpos"]
        gy = np.sum(dG * dval_dy, axis=0) * a["zpos"]
        g = M.ravel().astype(np.float64)
        X = np.arange(self.W, dtype=np.float64)[None, :]
        Y = np.arange(self.H, dtype=np.float64)[:, None]
        z = (g[6] * X + g[7] * Y) + g[8]
        x, y = a["x"], a["y"]
        with np.errstate(divide="ignore", invalid="ignore"):
            iz = np.where(a["zpos"], 1.0 / z, 0.0)
            terms = [gx * X * iz, gx * Y * iz, gx * iz, gy * X * iz, gy * Y * iz, gy * iz,
                     -(gx * x + gy * y) * X * iz, -(gx * x + gy * y) * Y * iz, -(gx * x + gy * y) * iz]
        dm = np.array([np.sum(np.where(a["zpos"], t, 0.0)) for t in terms]).reshape(3, 3)
        return df, dm

    def grad_q(self, q, H_fixed, w: int, h: int, frozen):
        """(loss, d loss / d q, d loss / d frames) with camera 0 fixed at H_fixed and
        camera 1 at H(q)."""
        H1 = dlt_from_corners(q, w, h)
        st = self.forward([H_fixed, H1], frozen)
        d_frames, d_M = self.backward(st)
        dH = canvas_map_jacobian(H1).T @ d_M[1].ravel()
        dq = dlt_jacobian(q, w, h).T @ dH
        return st["loss"], dq, d_frames


# ----------------------------------------------------------------------------- the whole path's VJP
class FrameVjpOracle:
    """The stitching path of any number of cameras as a function of FLOAT frames and the
    cameras' canvas -> source maps, R_0 = F(frames, M) (Alg. 4 steps 1 and 6, before
    quantisation), and its vector-Jacobian product: given an upstream dl/dR_0 (and
    optionally a direct dl/dG_0 per camera, a term on the warped frame itself), the
    gradients dl/dframe_i and dl/dM_i.

    Readings: the maps are the FP32 normalised inverses of the source -> canvas homographies
    (R3, 'spec') or their FP64 values ('ideal'); the bilinear cell is floor of the source
    coordinates at the given maps (at integers the right derivative), fixed while
    differentiating; every array lives on the full canvas (R12); masks are the plan's uint8
    seam weights (R9).  Transposes scatter every tap back with np.add.at, as GradOracle."""

    def __init__(self, frames, Hs, masks, canvas_w: int, canvas_h: int, levels: int, coords: str = "spec"):
        self.frames = [np.asarray(f, dtype=np.float64) for f in frames]
        self.Hs = [np.asarray(h, dtype=np.float64) for h in Hs]
        self.masks = [np.asarray(m, dtype=np.uint8) for m in masks]
        self.W, self.H, self.L = canvas_w, canvas_h, levels
        self.dims = level_dims(canvas_h, canvas_w, levels)
        self.coords = coords
        self.gm = []
        for m in self.masks:
            g = [m[None].astype(np.float64) / 255.0]
            for _ in range(levels - 1):
                g.append(reduce_full(g[-1]))
            self.gm.append(g)
        self.M = [hinv_ideal(h).astype(np.float32) if coords == "spec" else hinv_ideal(h) for h in self.Hs]
        self.cells = [self._cell(M) for M in self.M]

    def _coords(self, M):
        ft = np.float32 if M.dtype == np.float32 else np.float64
        g = M.ravel().astype(ft)
        X = np.arange(self.W, dtype=ft)[None, :]
        Y = np.arange(self.H, dtype=ft)[:, None]
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            u = (g[0] * X + g[1] * Y) + g[2]
            v = (g[3] * X + g[4] * Y) + g[5]
            z = (g[6] * X + g[7] * Y) + g[8]
            x = u / z
            y = v / z
        return x, y, z.astype(np.float64) > 0      # x, y in the maps' precision

    def _cell(self, M):
        x, y, zpos = self._coords(M)
        ok = zpos & np.isfinite(x) & np.isfinite(y) & (np.abs(x) < 1e7) & (np.abs(y) < 1e7)
        with np.errstate(invalid="ignore"):
            x0 = np.where(ok, np.floor(np.where(ok, x, 0.0)), -10).astype(np.int64)
            y0 = np.where(ok, np.floor(np.where(ok, y, 0.0)), -10).astype(np.int64)
        return x0, y0, ok

    def _warp(self, f, M, cell):
        """G_0 of a float frame through M with the fixed cell; taps outside count 0."""
        h, w = f.shape[1:]
        x, y, _ = self._coords(M)
        x0, y0, ok = cell
        # the fraction in the coordinates' precision, as the forward path takes it (R3):
        # for -1 < x < 0 the FP32 difference x - (-1) is rounded
        with np.errstate(invalid="ignore", over="ignore"):
            fx = np.where(ok, (x - x0.astype(x.dtype)).astype(np.float64), 0.0)
            fy = np.where(ok, (y - y0.astype(y.dtype)).astype(np.float64), 0.0)
        x, y = x.astype(np.float64), y.astype(np.float64)
        taps, okt = [], []
        for dy, dx in ((0, 0), (0, 1), (1, 0), (1, 1)):
            yy, xx = y0 + dy, x0 + dx
            k = ok & (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
            taps.append(np.where(k[None], f[:, np.clip(yy, 0, h - 1), np.clip(xx, 0, w - 1)], 0.0))
            okt.append(k)
        val = (1 - fy) * ((1 - fx) * taps[0] + fx * taps[1]) + fy * ((1 - fx) * taps[2] + fx * taps[3])
        return val, dict(x=x, y=y, fx=fx, fy=fy, ok=ok, taps=taps, okt=okt)

    def _collapse_of(self, G0s):
        laps = []
        for g in G0s:
            gp = [g]
            for _ in range(self.L - 1):
                gp.append(reduce_full(gp[-1]))
            laps.append([gp[k] - expand_full(gp[k + 1], *gp[k].shape[-2:]) for k in range(self.L - 1)] + [gp[-1]])
        B = [sum(self.gm[i][k] * laps[i][k] for i in range(len(G0s))) for k in range(self.L)]
        R = B[-1]
        for k in range(self.L - 2, -1, -1):
            R = B[k] + expand_full(R, *B[k].shape[-2:])
        return R

    def forward(self, frames=None, maps=None):
        """R_0 (3, H, W) of the float frames through the maps (default: the object's own),
        with the cells fixed at the object's maps."""
        frames = self.frames if frames is None else [np.asarray(f, dtype=np.float64) for f in frames]
        maps = self.M if maps is None else maps
        return self._collapse_of([self._warp(f, M, c)[0] for f, M, c in zip(frames, maps, self.cells)])

    def vjp(self, dR0, dG0=None):
        """(d_frames, d_M) for the upstream gradient dR0 (3, H, W) and optional direct
        gradients dG0[i] (3, H, W) on the warped frames."""
        L = self.L
        dR = [np.asarray(dR0, dtype=np.float64)]
        for _ in range(L - 1):
            dR.append(expand_T(dR[-1]))
        d_frames, d_M = [], []
        for i, f in enumerate(self.frames):
            dL = [self.gm[i][k] * dR[k] for k in range(L)]
            if L == 1:
                dG = dL[0]
            else:
                g = dL[L - 1] - expand_T(dL[L - 2])
                for k in range(L - 2, 0, -1):
                    g = dL[k] - expand_T(dL[k - 1]) + reduce_T(g, *self.dims[k])
                dG = dL[0] + reduce_T(g, *self.dims[0])
            if dG0 is not None and dG0[i] is not None:
                dG = dG + dG0[i]
            df, dm = self._warp_T(f, self.M[i], self.cells[i], dG)
            d_frames.append(df)
            d_M.append(dm)
        return d_frames, d_M

    def _warp_T(self, f, M, cell, dG):
        h, w = f.shape[1:]
        _, a = self._warp(f, M, cell)
        x0, y0, ok = cell
        fx, fy = a["fx"], a["fy"]
        wts = [(1 - fy) * (1 - fx), (1 - fy) * fx, fy * (1 - fx), fy * fx]
        df = np.zeros_like(f)
        for wt, (dy, dx), k in zip(wts, ((0, 0), (0, 1), (1, 0), (1, 1)), a["okt"]):
            for c in range(3):
                np.add.at(df[c], ((y0 + dy)[k], (x0 + dx)[k]), (wt * dG[c])[k])
        p00, p01, p10, p11 = a["taps"]
        gx = np.sum(dG * ((1 - fy) * (p01 - p00) + fy * (p11 - p10)), axis=0) * ok
        gy = np.sum(dG * ((1 - fx) * (p10 - p00) + fx * (p11 - p01)), axis=0) * ok
        g = M.ravel().astype(np.float64)
        X = np.arange(self.W, dtype=np.float64)[None, :]
        Y = np.arange(self.H, dtype=np.float64)[:, None]
        z = (g[6] * X + g[7] * Y) + g[8]
        x, y = a["x"], a["y"]
        with np.errstate(divide="ignore", invalid="ignore"):
            iz = np.where(ok, 1.0 / z, 0.0)
            s = -(gx * np.where(ok, x, 0.0) + gy * np.where(ok, y, 0.0)) * iz
            terms = [gx * X * iz, gx * Y * iz, gx * iz, gy * X * iz, gy * Y * iz, gy * iz, s * X, s * Y, s]
        dm = np.array([np.sum(np.where(ok, t, 0.0)) for t in terms]).reshape(3, 3)
        return df, dm
