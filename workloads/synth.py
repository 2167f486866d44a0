"""Synthetic rigs and frames for the per-frame stitching path.

The paper's captured videos (2304x1728, Sec. 5) and its rig calibration are not
available, so every input here is seeded and synthetic, with the shapes of the
paper's workloads: several cameras facing different directions whose frames
overlap (Alg. 4 input), fixed "pre-corrected" homographies (Alg. 4, step 1),
and one panoramic canvas.

Scene: one analytic texture per job, defined on canvas coordinates, so that the
overlaps of different cameras agree.  Per channel c

    S_c(X, Y) = 0.5 + 0.4 * (1/8) * sum_j sin(2 pi f_j (X cos t_j + Y sin t_j) + p_j)

with t_j ~ U[0, pi), f_j ~ U[1/64, 1/8] cycles/px, p_j ~ U[0, 2 pi).  Camera i's
pixel (x, y) sees S at H_i(x, y) (H_i maps source -> canvas), plus uniform noise
U[-0.05, 0.05], and is quantised as rint(255 * clip(t, 0, 1)).

Noise comes from a counter-based 32-bit integer hash evaluated with exact int64
tensor arithmetic, so the same seed gives the same bytes on the CPU and on a GPU.
The scene itself is evaluated in float64 with torch.sin on the chosen device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

ROOT_SEED = 181003988
TAG_SCENE, TAG_NOISE, TAG_GEOM = 0, 1, 2


def _seq(config: int, job: int, camera: int, frame: int, tag: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([ROOT_SEED, config, job, camera, frame, tag])


def _key32(config: int, job: int, camera: int, frame: int, tag: int) -> tuple[int, int]:
    w = _seq(config, job, camera, frame, tag).generate_state(2, dtype=np.uint32)
    return int(w[0]), int(w[1])


# ----------------------------------------------------------------------------- noise
_M32 = 0xFFFFFFFF


def _mul32(x: torch.Tensor, c: int) -> torch.Tensor:
    """(x * c) mod 2^32 for 0 <= x < 2^32, with every intermediate below 2^63."""
    lo = x * (c & 0xFFFF)
    hi = ((x * (c >> 16)) & 0xFFFF) << 16
    return (lo + hi) & _M32


def _hash32(x: torch.Tensor) -> torch.Tensor:
    """A 32-bit integer finaliser (xorshift-multiply, constants 0x7feb352d and
    0x846ca68b, shifts 16/15/16) on int64 tensors holding values < 2^32."""
    x = x ^ (x >> 16)
    x = _mul32(x, 0x7FEB352D)
    x = x ^ (x >> 15)
    x = _mul32(x, 0x846CA68B)
    x = x ^ (x >> 16)
    return x


def hash32_noise(n: int, key: tuple[int, int], device="cpu") -> torch.Tensor:
    """n samples of U[-0.05, 0.05) (float64) from counters 0..n-1 under a 64-bit key."""
    idx = torch.arange(n, dtype=torch.int64, device=device)
    h = _hash32(_hash32((idx & _M32) ^ key[0]) ^ ((idx >> 32) ^ key[1]))
    return h.to(torch.float64) * (0.1 / 4294967296.0) - 0.05


# ----------------------------------------------------------------------------- scene
def scene_params(config: int, job: int) -> np.ndarray:
    """(3 channels, 3 [theta, f, phi], 8 sinusoids) float64."""
    rng = np.random.default_rng(_seq(config, job, 0, 0, TAG_SCENE))
    out = np.empty((3, 3, 8))
    for c in range(3):
        out[c, 0] = rng.uniform(0.0, math.pi, 8)
        out[c, 1] = rng.uniform(1.0 / 64.0, 1.0 / 8.0, 8)
        out[c, 2] = rng.uniform(0.0, 2.0 * math.pi, 8)
    return out


def scene_values(params: np.ndarray, H: np.ndarray, w: int, h: int, device="cpu") -> torch.Tensor:
    """Noise-free scene seen by a (w x h) camera through H (source -> canvas): (h, w, 3) float64."""
    Ht = torch.as_tensor(np.asarray(H, dtype=np.float64), device=device)
    pr = torch.as_tensor(params, device=device)
    ys = torch.arange(h, dtype=torch.float64, device=device)
    xs = torch.arange(w, dtype=torch.float64, device=device)
    y, x = torch.meshgrid(ys, xs, indexing="ij")
    zc = Ht[2, 0] * x + Ht[2, 1] * y + Ht[2, 2]
    X = (Ht[0, 0] * x + Ht[0, 1] * y + Ht[0, 2]) / zc
    Y = (Ht[1, 0] * x + Ht[1, 1] * y + Ht[1, 2]) / zc
    del x, y, zc
    out = torch.empty((h, w, 3), dtype=torch.float64, device=device)
    for c in range(3):
        acc = torch.zeros_like(X)
        for j in range(8):
            th, f, ph = pr[c, 0, j], pr[c, 1, j], pr[c, 2, j]
            acc += torch.sin(2.0 * math.pi * f * (X * torch.cos(th) + Y * torch.sin(th)) + ph)
        out[..., c] = 0.5 + 0.4 * acc / 8.0
    return out


def quantise_with_noise(scene: torch.Tensor, key: tuple[int, int]) -> torch.Tensor:
    """rint(255 * clip(scene + U[-0.05, 0.05], 0, 1)) as uint8, noise keyed per frame."""
    noise = hash32_noise(scene.numel(), key, scene.device).view(scene.shape)
    return torch.round(255.0 * (scene + noise).clamp(0.0, 1.0)).to(torch.uint8)


def render_frames(params: np.ndarray, H: np.ndarray, w: int, h: int, key: tuple[int, int],
                  device="cpu") -> torch.Tensor:
    """Render one camera frame (h, w, 3) uint8 seeing the scene through H (source -> canvas)."""
    return quantise_with_noise(scene_values(params, H, w, h, device), key)


# ----------------------------------------------------------------------------- geometry
def _T(tx: float, ty: float) -> np.ndarray:
    return np.array([[1.0, 0.0, tx], [0.0, 1.0, ty], [0.0, 0.0, 1.0]])


def _Rz(deg: float) -> np.ndarray:
    a = math.radians(deg)
    return np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])


def _Ry(deg: float) -> np.ndarray:
    a = math.radians(deg)
    return np.array([[math.cos(a), 0.0, math.sin(a)], [0.0, 1.0, 0.0], [-math.sin(a), 0.0, math.cos(a)]])


def _K(f: float, cx: float, cy: float) -> np.ndarray:
    return np.array([[f, 0.0, cx], [0.0, f, cy], [0.0, 0.0, 1.0]])


def seam_masks(canvas_w: int, canvas_h: int, seams: list[int]) -> list[np.ndarray]:
    """Binary vertical cuts: camera i owns columns [s_{i-1}, s_i) with s_{-1}=0, s_{n-1}=W.
    Returned as uint8 weights (255 owned, 0 elsewhere); they sum to 255 everywhere."""
    bounds = [0] + list(seams) + [canvas_w]
    masks = []
    for i in range(len(bounds) - 1):
        m = np.zeros((canvas_h, canvas_w), dtype=np.uint8)
        m[:, bounds[i]:bounds[i + 1]] = 255
        masks.append(m)
    return masks


@dataclass
class Rig:
    """A fixed camera rig: frame sizes, source->canvas homographies, canvas, seams, levels."""
    name: str
    config: int
    job: int
    frame_sizes: list            # [(w, h)] per camera
    H: list                      # [3x3 float64] per camera, source -> canvas
    canvas_w: int
    canvas_h: int
    levels: int
    seams: list                  # n-1 vertical cut columns
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.H)

    def masks(self) -> list[np.ndarray]:
        return seam_masks(self.canvas_w, self.canvas_h, self.seams)

    def canvas_pixels(self) -> int:
        return self.canvas_w * self.canvas_h


def rig_ring(name, config, job, n, w, h, centres_x, yaws_deg, focal, canvas_w, canvas_h, levels) -> Rig:
    """Cameras with small residual yaws (keystones) placed along a horizontal canvas.

    H_i = T(o_i, oy) K R_y(yaw_i) K^-1, with o_i chosen so the frame centre lands at
    centres_x[i]; seams at the rounded-up midpoints of the translation-only overlaps."""
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    K = _K(focal, cx, cy)
    Ki = np.linalg.inv(K)
    oy = (canvas_h - h) / 2.0
    Hs, lefts, rights = [], [], []
    for i in range(n):
        shift = focal * math.tan(math.radians(yaws_deg[i]))
        Hi = _T(centres_x[i] - cx - shift, oy) @ K @ _Ry(yaws_deg[i]) @ Ki
        Hs.append(Hi / Hi[2, 2])
        lefts.append(centres_x[i] - cx)
        rights.append(centres_x[i] + cx)
    seams = [int(math.ceil((lefts[i + 1] + rights[i]) / 2.0)) for i in range(n - 1)]
    return Rig(name, config, job, [(w, h)] * n, Hs, canvas_w, canvas_h, levels, seams,
               extra={"yaws_deg": list(yaws_deg), "focal": focal, "centres_x": list(centres_x)})


def rig_c1() -> Rig:
    """Two 640x480 frames; A identity, B = T(400,3) about-centre 2 degree rotation; 1040x480, L=5."""
    c = (319.5, 239.5)
    HB = _T(400.0, 3.0) @ _T(*c) @ _Rz(2.0) @ _T(-c[0], -c[1])
    return Rig("C1", 1, 0, [(640, 480), (640, 480)], [np.eye(3), HB], 1040, 480, 5, [520])


def _ring_centres(n, mid, spacing):
    return [mid + (i - (n - 1) / 2.0) * spacing for i in range(n)]


def rig_c2() -> Rig:
    """Four 1920x1080 cameras, residual yaws -3,-1,+1,+3 degrees, f=1100, 6400x1080 canvas, L=6."""
    return rig_ring("C2", 2, 0, 4, 1920, 1080, _ring_centres(4, 3199.5, 1632.0), [-3.0, -1.0, 1.0, 3.0],
                    1100.0, 6400, 1080, 6)


def rig_c4() -> Rig:
    """C2 scaled by two: four 3840x2160 cameras, f=2200, 12800x2160 canvas, L=7."""
    return rig_ring("C4", 4, 0, 4, 3840, 2160, _ring_centres(4, 6399.5, 3264.0), [-3.0, -1.0, 1.0, 3.0],
                    2200.0, 12800, 2160, 7)


C3_RESOLUTIONS = [(640, 480), (1280, 720), (1920, 1080), (3840, 2160)]


def rig_c3_jobs(njobs: int = 64, resolutions=None) -> list[Rig]:
    """Heterogeneous stitch jobs: 2..6 cameras, one resolution per job, 10-25% overlaps,
    residual yaws spread over [-3, 3] degrees, L = floor(log2(min side)) - 4."""
    resolutions = resolutions or C3_RESOLUTIONS
    rigs = []
    for j in range(njobs):
        rng = np.random.default_rng(_seq(3, j, 0, 0, TAG_GEOM))
        n = int(rng.integers(2, 7))
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        r = float(rng.uniform(0.10, 0.25))
        W = int(math.ceil(w + (n - 1) * (1.0 - r) * w))
        centres = [(w - 1) / 2.0 + i * (1.0 - r) * w for i in range(n)]
        yaws = [-3.0 + 6.0 * i / (n - 1) for i in range(n)]
        L = int(math.floor(math.log2(min(w, h)))) - 4
        rigs.append(rig_ring(f"C3.job{j}", 3, j, n, w, h, centres, yaws, 1100.0 * w / 1920.0, W, h, L))
    return rigs


def rig_c5_pairs(npairs: int = 16) -> list[Rig]:
    """Pairs of 1280x720 frames with 20% overlap on a 2304x720 canvas, L=3.

    H_A = I; the ground-truth H_B = T(1024,0) K R_y(phi) K^-1 with phi ~ U[-2, 2] degrees
    and f = 733.3.  extra["corner_noise"] holds U[-3, 3] px offsets for B's four corners."""
    rigs = []
    w, h, f = 1280, 720, 733.3
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    K = _K(f, cx, cy)
    Ki = np.linalg.inv(K)
    for p in range(npairs):
        rng = np.random.default_rng(_seq(5, p, 0, 0, TAG_GEOM))
        phi = float(rng.uniform(-2.0, 2.0))
        HB = _T(1024.0, 0.0) @ K @ _Ry(phi) @ Ki
        HB = HB / HB[2, 2]
        noise = rng.uniform(-3.0, 3.0, 8)
        rigs.append(Rig(f"C5.pair{p}", 5, p, [(w, h), (w, h)], [np.eye(3), HB], 2304, 720, 3, [1152],
                        extra={"yaw_deg": phi, "corner_noise": noise}))
    return rigs


def render_rig_frames(rig: Rig, frame: int = 0, device="cpu") -> list[torch.Tensor]:
    """All camera frames of one rig at one time step (noise reseeded per frame)."""
    return render_rig_sequence(rig, [frame], device)[0]


def render_rig_sequence(rig: Rig, frames, device="cpu") -> list[list[torch.Tensor]]:
    """Frames of a fixed rig over time: same scene and H, noise reseeded per frame index.
    Returns out[t][camera] as (h, w, 3) uint8 tensors."""
    params = scene_params(rig.config, rig.job)
    frames = list(frames)
    out = [[None] * rig.n for _ in frames]
    for i, ((w, h), H) in enumerate(zip(rig.frame_sizes, rig.H)):
        scene = scene_values(params, H, w, h, device)
        for t, f in enumerate(frames):
            out[t][i] = quantise_with_noise(scene, _key32(rig.config, rig.job, i, f, TAG_NOISE))
        del scene
    return out


# ----------------------------------------------------------------------------- feature-extraction inputs
def brief_pattern(nd: int = 256, seed: int = 0) -> np.ndarray:
    """n_d point pairs for a BRIEF descriptor as an (nd, 4) int32 array of offsets
    (dx1, dy1, dx2, dy2), each drawn from an isotropic Gaussian of sigma 31/5 around the
    point, rounded and clipped to the 31x31 patch (|d| <= 15).  Input data only."""
    rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 90, seed]))
    d = np.rint(rng.normal(0.0, 31.0 / 5.0, size=(nd, 4)))
    return np.clip(d, -15, 15).astype(np.int32)


def rotated_frame(frame: np.ndarray, deg: float) -> np.ndarray:
    """The (h, w, 3) uint8 frame turned by deg about its centre, nearest sample, 0 outside:
    the synthetic rotations the BRIEF descriptor is probed with (Fig. 2).  Input data only."""
    h, w = frame.shape[:2]
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    c, s = np.cos(np.radians(deg)), np.sin(np.radians(deg))
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    sx = np.rint(c * (x - cx) + s * (y - cy) + cx).astype(np.int64)
    sy = np.rint(-s * (x - cx) + c * (y - cy) + cy).astype(np.int64)
    ok = (sx >= 0) & (sx < w) & (sy >= 0) & (sy < h)
    out = np.zeros_like(frame)
    out[ok] = frame[sy[ok], sx[ok]]
    return out
