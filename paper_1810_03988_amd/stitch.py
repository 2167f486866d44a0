"""ctypes binding of libstitch.so: argument marshalling only.

Torch tensors supply device memory (data_ptr) and the stream
(torch.cuda.current_stream().cuda_stream); every step of the path runs in the HIP
kernels behind the C ABI.  There is no fallback: if the library is missing or a call
fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint8, c_void_p
from pathlib import Path

import numpy as np
import torch

# the in-tree build; STITCH_LIB names another build of the same sources (the host-sanitized
# one the ABI tests use), never a substitute for the HIP kernels
LIB_PATH = Path(os.environ.get("STITCH_LIB") or Path(__file__).resolve().with_name("libstitch.so"))

U8, F16, F32 = 0, 1, 2
HWC, CHW = 0, 1
MAX_LEVELS = 16
KEEP_R0 = 1
STATUS = ["OK", "E_NULL", "E_SHAPE", "E_LEVELS", "E_HOMOGRAPHY", "E_MASK", "E_WORKSPACE", "E_DEVICE",
          "E_UNSUPPORTED", "E_STATE"]


class StitchImage(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("width", c_int32), ("height", c_int32), ("channels", c_int32),
                ("dtype", c_int32), ("layout", c_int32), ("row_pitch", c_int64), ("plane_pitch", c_int64)]


class StitchLevels(ctypes.Structure):
    _fields_ = [("levels", c_int32), ("canvas_w", c_int32), ("canvas_h", c_int32),
                ("origin_x", c_int32 * MAX_LEVELS), ("origin_y", c_int32 * MAX_LEVELS),
                ("level", StitchImage * MAX_LEVELS)]


class MatchPair(ctypes.Structure):
    """One area pair of stitch_lsh_match_multi (stitch_match_pair): device pointers."""
    _fields_ = [("desc_a", c_void_p), ("count_a", c_void_p), ("cap_a", c_int32), ("desc_b", c_void_p),
                ("count_b", c_void_p), ("cap_b", c_int32), ("match", c_void_p), ("dist", c_void_p)]


class ProsacPair(ctypes.Structure):
    """One area pair of stitch_prosac_multi (stitch_prosac_pair): device pointers."""
    _fields_ = [("pts_a", c_void_p), ("pts_b", c_void_p), ("cap_b", c_int32), ("match", c_void_p),
                ("dist", c_void_p), ("count_a", c_void_p), ("cap_a", c_int32), ("uniforms", c_void_p),
                ("H", c_void_p), ("inliers", c_void_p), ("inlier_mask", c_void_p), ("hyp_counts", c_void_p)]


class StitchError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"stitch {name}: {message}")


_lib = None

# name -> (restype, argtypes); every symbol of include/stitch.h
SIGNATURES = {
    "stitch_abi_version": (c_int32, []),
    "stitch_status_str": (c_char_p, [c_int32]),
    "stitch_last_error": (c_char_p, []),
    "stitch_warp": (c_int32, [POINTER(StitchImage), POINTER(c_double), c_int32, c_int32, POINTER(StitchImage),
                              c_void_p]),
    "stitch_warp_coords": (c_int32, [POINTER(c_double), c_int32, c_int32, POINTER(StitchImage), c_void_p]),
    "stitch_pyramid_workspace_bytes": (c_size_t, [c_int32]),
    "stitch_pyramid": (c_int32, [POINTER(StitchImage), c_int32, POINTER(StitchLevels), c_void_p, c_size_t,
                                 c_void_p]),
    "stitch_blend_workspace_bytes": (c_size_t, [c_int32, c_int32]),
    "stitch_blend": (c_int32, [c_int32, POINTER(StitchLevels), POINTER(StitchLevels), POINTER(StitchImage),
                               POINTER(StitchLevels), c_void_p, c_size_t, c_void_p]),
    "stitch_plan_create": (c_int32, [c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_double),
                                     POINTER(POINTER(c_uint8)), c_int32, c_int32, c_int32, c_int32, c_int32,
                                     POINTER(c_void_p)]),
    "stitch_plan_workspace_bytes": (c_size_t, [c_void_p]),
    "stitch_plan_bind": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "stitch_frame": (c_int32, [c_void_p, POINTER(StitchImage), POINTER(StitchImage), c_void_p]),
    "stitch_plan_view": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(StitchImage), POINTER(c_int32),
                                   POINTER(c_int32)]),
    "stitch_plan_regions": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "stitch_plan_set_timing": (c_int32, [c_void_p, c_int32]),
    "stitch_plan_read_timing": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int32)]),
    "stitch_plan_destroy": (None, [c_void_p]),
    "stitch_batch_create": (c_int32, [c_int32, POINTER(c_void_p), POINTER(c_void_p)]),
    "stitch_batch_workspace_bytes": (c_size_t, [c_void_p]),
    "stitch_batch_bind": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "stitch_batch_run": (c_int32, [c_void_p, POINTER(POINTER(StitchImage)), POINTER(StitchImage), c_void_p]),
    "stitch_batch_autotune": (c_int32, [c_void_p, POINTER(POINTER(StitchImage)), POINTER(StitchImage), c_void_p,
                                        c_char_p]),
    "stitch_batch_config": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "stitch_batch_set_config": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "stitch_batch_set_groups": (c_int32, [c_void_p, c_int32]),
    "stitch_batch_group_count": (c_int32, [c_void_p]),
    "stitch_plan_config": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "stitch_plan_set_config": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), c_void_p]),
    "stitch_autotune": (c_int32, [c_void_p, POINTER(StitchImage), c_void_p, c_char_p]),
    "stitch_batch_set_timing": (c_int32, [c_void_p, c_int32]),
    "stitch_batch_read_timing": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int32)]),
    "stitch_batch_destroy": (None, [c_void_p]),
    "stitch_grad_create": (c_int32, [POINTER(c_int32), POINTER(c_int32), POINTER(POINTER(c_uint8)), c_int32,
                                     c_int32, c_int32, POINTER(c_void_p)]),
    "stitch_grad_workspace_bytes": (c_size_t, [c_void_p]),
    "stitch_grad_bind": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "stitch_grad_freeze": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64), c_void_p]),
    "stitch_grad_forward": (c_int32, [c_void_p, POINTER(StitchImage), POINTER(c_double), POINTER(c_double),
                                      c_void_p]),
    "stitch_grad_backward": (c_int32, [c_void_p, POINTER(StitchImage), POINTER(c_double), c_void_p]),
    "stitch_grad_upstream": (c_int32, [c_void_p, POINTER(StitchImage), POINTER(StitchImage), c_void_p]),
    "stitch_grad_destroy": (None, [c_void_p]),
    "stitch_pipe_workspace_bytes": (c_size_t, [c_void_p, c_int32]),
    "stitch_pipe_create": (c_int32, [c_void_p, c_int32, c_void_p, c_size_t, POINTER(c_void_p)]),
    "stitch_pipe_run": (c_int32, [c_void_p, c_int32, POINTER(c_void_p), POINTER(c_void_p)]),
    "stitch_pipe_destroy": (None, [c_void_p]),
    "stitch_host_alloc": (c_int32, [c_size_t, POINTER(c_void_p)]),
    "stitch_host_free": (None, [c_void_p]),
    "stitch_frame_backward_workspace_bytes": (c_size_t, [c_void_p]),
    "stitch_frame_forward_f32": (c_int32, [c_void_p, POINTER(StitchImage), POINTER(StitchImage), c_void_p, c_size_t,
                                           c_void_p]),
    "stitch_frame_backward": (c_int32, [c_void_p, POINTER(StitchImage), POINTER(StitchImage), POINTER(StitchImage),
                                        POINTER(StitchImage), POINTER(c_double), c_void_p, c_size_t, c_void_p]),
    "stitch_corners_to_h": (c_int32, [POINTER(c_double), c_int32, c_int32, POINTER(c_double)]),
    "stitch_map_grad_to_corners": (c_int32, [POINTER(c_double), c_int32, c_int32, POINTER(c_double),
                                             POINTER(c_double)]),
    "stitch_lorb_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32, POINTER(c_int32)]),
    "stitch_lorb": (c_int32, [POINTER(StitchImage), c_int32, POINTER(c_int32), c_int32, c_int64, c_int32, c_int32,
                              c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "stitch_lorb_set_timing": (c_int32, [c_int32]),
    "stitch_detection_areas": (c_int32, [c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_double), c_int32,
                                         c_int32, c_int32, c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "stitch_lorb_multi_workspace_bytes": (c_size_t, [c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                                     POINTER(c_int32)]),
    "stitch_lorb_multi": (c_int32, [c_int32, POINTER(StitchImage), POINTER(c_int32), POINTER(c_int32), c_int32,
                                    c_int64, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_size_t, c_void_p]),
    "stitch_lsh_match_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32]),
    "stitch_lsh_match": (c_int32, [c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_int32,
                                   c_int32, POINTER(c_int32), c_int32, c_void_p, c_void_p, c_void_p, c_size_t,
                                   c_void_p]),
    "stitch_prosac_workspace_bytes": (c_size_t, [c_int32, c_int32]),
    "stitch_prosac": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                c_void_p, c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_size_t, c_void_p]),
    "stitch_lorb_read_timing": (c_int32, [POINTER(c_double), POINTER(c_int32)]),
    "stitch_prosac_noalloc": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                        c_void_p, c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p]),
    "stitch_lsh_match_multi_workspace_bytes": (c_size_t, [c_int32, POINTER(MatchPair), c_int32]),
    "stitch_lsh_match_multi": (c_int32, [c_int32, POINTER(MatchPair), c_int32, c_int32, c_int32, POINTER(c_int32),
                                         c_int32, c_void_p, c_size_t, c_void_p]),
    "stitch_prosac_multi_workspace_bytes": (c_size_t, [c_int32, POINTER(ProsacPair), c_int32]),
    "stitch_prosac_multi": (c_int32, [c_int32, POINTER(ProsacPair), c_int32, c_double, c_double, c_void_p,
                                      c_size_t, c_void_p]),
}

TIMING_KINDS = ["warp_level0_pass", "level_pass", "blend_level0", "blend_middle", "blend_top",
                "blend_single", "warp_single", "unused"]


def lib():
    """Load libstitch.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1810_03988_amd.build` "
                              "(or __graft_entry__.build()); there is no fallback path")
        handle = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int) -> None:
    if status != 0:
        raise StitchError(status, lib().stitch_last_error().decode())


def last_error() -> str:
    return lib().stitch_last_error().decode()


# ----------------------------------------------------------------------------- marshalling
_DT = {torch.uint8: U8, torch.float16: F16, torch.float32: F32}
_TORCH_DT = {U8: torch.uint8, F16: torch.float16, F32: torch.float32}


def _on_gpu(t: torch.Tensor, name: str) -> None:
    """Every pointer the device calls take must be device memory: a host tensor's address
    handed to a kernel would fault, so it is refused before any launch."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (got {getattr(t, 'device', type(t))})")


def image_hwc(t: torch.Tensor) -> StitchImage:
    """(H, W, C) GPU tensor with unit channel stride -> HWC image view."""
    _on_gpu(t, "image")
    if t.dim() != 3 or t.stride(2) != 1 or t.stride(1) != t.shape[2]:
        raise ValueError("HWC images need shape (H, W, C) with packed pixels")
    es = t.element_size()
    return StitchImage(t.data_ptr(), t.shape[1], t.shape[0], t.shape[2], _DT[t.dtype], HWC, t.stride(0) * es, 0)


def image_chw(t: torch.Tensor) -> StitchImage:
    """(C, H, W) or (H, W) GPU tensor with unit column stride -> CHW image view."""
    _on_gpu(t, "image")
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3 or t.stride(2) != 1:
        raise ValueError("CHW images need shape (C, H, W) with unit column stride")
    es = t.element_size()
    return StitchImage(t.data_ptr(), t.shape[2], t.shape[1], t.shape[0], _DT[t.dtype], CHW, t.stride(1) * es,
                       t.stride(0) * es)


def levels_struct(levels: list, origins: list, canvas_w: int, canvas_h: int) -> StitchLevels:
    s = StitchLevels()
    s.levels = len(levels)
    s.canvas_w, s.canvas_h = canvas_w, canvas_h
    for k, t in enumerate(levels):
        if t is None:
            s.level[k] = StitchImage()
            continue
        s.level[k] = image_chw(t)
        s.origin_x[k], s.origin_y[k] = origins[k]
    return s


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _h9(H) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(9))
    return (c_double * 9)(*a.tolist())


def level_dims(canvas_h: int, canvas_w: int, levels: int) -> list:
    dims = [(canvas_h, canvas_w)]
    for _ in range(levels - 1):
        dims.append(((dims[-1][0] + 1) // 2, (dims[-1][1] + 1) // 2))
    return dims


# ----------------------------------------------------------------------------- single stages
def warp(src: torch.Tensor, H, roi_x: int, roi_y: int, width: int, height: int, dtype=torch.float32,
         out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """G_0 (3, height, width) of one camera over a canvas rectangle."""
    if out is None:
        out = torch.empty((3, height, width), dtype=dtype, device=src.device)
    check(lib().stitch_warp(ctypes.byref(image_hwc(src)), _h9(H), roi_x, roi_y, ctypes.byref(image_chw(out)),
                            _stream(stream)))
    return out


def warp_coords(H, roi_x: int, roi_y: int, width: int, height: int, device="cuda", stream=None) -> torch.Tensor:
    out = torch.empty((2, height, width), dtype=torch.float32, device=device)
    check(lib().stitch_warp_coords(_h9(H), roi_x, roi_y, ctypes.byref(image_chw(out)), _stream(stream)))
    return out


def pyramid(g0: torch.Tensor, levels: int, kind: str = "laplacian", canvas=None, origin=(0, 0),
            dtype=None, stream=None) -> list:
    """Gaussian or Laplacian pyramid of g0 ((C,H,W) float or (H,W) uint8 weights) placed at
    `origin` on a canvas of size `canvas` (w, h; default: g0's own size), stored on the
    rectangles [origin >> k, ceil((origin + size) / 2^k))."""
    if g0.dtype == torch.uint8 and g0.dim() == 2:
        g0v = g0.unsqueeze(0)
        dtype = dtype or torch.float32
    else:
        g0v = g0
        dtype = dtype or g0.dtype
    C, h, w = g0v.shape
    cw, ch = canvas if canvas is not None else (w, h)
    ox, oy = origin
    outs, origins = [], []
    for k in range(levels):
        x0, y0 = ox >> k, oy >> k
        x1 = min(-(-(ox + w) // (1 << k)), -(-cw // (1 << k)))
        y1 = min(-(-(oy + h) // (1 << k)), -(-ch // (1 << k)))
        outs.append(torch.empty((C, y1 - y0, x1 - x0), dtype=dtype, device=g0.device))
        origins.append((x0, y0))
    s = levels_struct(outs, origins, cw, ch)
    nbytes = lib().stitch_pyramid_workspace_bytes(levels)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=g0.device)
    base = (ws.data_ptr() + 255) // 256 * 256
    src = StitchImage(g0v.data_ptr(), w, h, C, _DT[g0v.dtype], CHW, g0v.stride(1) * g0v.element_size(),
                      g0v.stride(0) * g0v.element_size())
    check(lib().stitch_pyramid(ctypes.byref(src), 0 if kind.startswith("g") else 1, ctypes.byref(s), base, nbytes,
                               _stream(stream)))
    return outs


def blend(bands: list, weights: list, canvas_w: int, canvas_h: int, band_origins=None, weight_origins=None,
          keep_r: bool = True, stream=None):
    """Blend n Laplacian pyramids with n weight pyramids; returns (pano uint8 (H,W,3), R levels)."""
    n = len(bands)
    L = len(bands[0])
    dev = bands[0][0].device
    dt = bands[0][0].dtype
    zeros = [(0, 0)] * L
    band_origins = band_origins or [zeros] * n
    weight_origins = weight_origins or [zeros] * n
    bs = (StitchLevels * n)(*[levels_struct(b, o, canvas_w, canvas_h) for b, o in zip(bands, band_origins)])
    ws_ = (StitchLevels * n)(*[levels_struct(w, o, canvas_w, canvas_h) for w, o in zip(weights, weight_origins)])
    pano = torch.empty((canvas_h, canvas_w, 3), dtype=torch.uint8, device=dev)
    rs = [torch.empty((3, h, w), dtype=dt, device=dev) for h, w in level_dims(canvas_h, canvas_w, L)]
    if not keep_r:
        rs[0] = None
    rstruct = levels_struct(rs, zeros, canvas_w, canvas_h)
    nbytes = lib().stitch_blend_workspace_bytes(n, L)
    wsp = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = (wsp.data_ptr() + 255) // 256 * 256
    check(lib().stitch_blend(n, bs, ws_, ctypes.byref(image_hwc(pano)), ctypes.byref(rstruct), base, nbytes,
                             _stream(stream)))
    return pano, rs


# ----------------------------------------------------------------------------- planned frame path
class Plan:
    """A fixed rig planned once (Sec. 4.3.2 pre-allocation): validation, per-camera
    regions and the workspace, then stitch_frame per frame set."""

    def __init__(self, frame_sizes, Hs, masks, canvas_w: int, canvas_h: int, levels: int,
                 storage: str = "f32", keep_r0: bool = False, device="cuda", bind: bool = True):
        L = lib()
        n = len(Hs)
        self.n, self.canvas_w, self.canvas_h, self.levels = n, canvas_w, canvas_h, levels
        self.storage = F16 if storage in ("f16", torch.float16, F16) else F32
        self.frame_sizes = [tuple(map(int, s)) for s in frame_sizes]
        fw = (c_int32 * n)(*[s[0] for s in self.frame_sizes])
        fh = (c_int32 * n)(*[s[1] for s in self.frame_sizes])
        Hflat = np.ascontiguousarray(np.stack([np.asarray(h, dtype=np.float64).reshape(9) for h in Hs]))
        self._masks = [np.ascontiguousarray(np.asarray(m, dtype=np.uint8)) for m in masks]
        for m in self._masks:
            if m.shape != (canvas_h, canvas_w):
                raise ValueError("each mask must be (canvas_h, canvas_w) uint8")
        mptrs = (POINTER(c_uint8) * n)(*[m.ctypes.data_as(POINTER(c_uint8)) for m in self._masks])
        handle = c_void_p()
        check(L.stitch_plan_create(n, fw, fh, Hflat.ctypes.data_as(POINTER(c_double)), mptrs, canvas_w, canvas_h,
                                   levels, self.storage, KEEP_R0 if keep_r0 else 0, ctypes.byref(handle)))
        self._h = handle
        self._masks = None   # the plan keeps its own copy
        self.ws_bytes = L.stitch_plan_workspace_bytes(self._h)
        self.device = torch.device(device)
        self.workspace = None
        if bind:
            self.bind()

    def bind(self, workspace: torch.Tensor | None = None, stream=None) -> None:
        if workspace is None:
            workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = (workspace.data_ptr() + 255) // 256 * 256
        check(lib().stitch_plan_bind(self._h, base, self.ws_bytes, _stream(stream)))
        self.workspace = workspace
        self._base = base

    def frame(self, frames, pano: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if pano is None:
            pano = torch.empty((self.canvas_h, self.canvas_w, 3), dtype=torch.uint8, device=frames[0].device)
        fr = (StitchImage * self.n)(*[image_hwc(f) for f in frames])
        check(lib().stitch_frame(self._h, fr, ctypes.byref(image_hwc(pano)), _stream(stream)))
        return pano

    def frame_args(self, frames, pano):
        """Pre-marshalled arguments for repeated stitch_frame calls (timing loops)."""
        fr = (StitchImage * self.n)(*[image_hwc(f) for f in frames])
        return fr, image_hwc(pano)

    def frame_raw(self, args, stream_handle: int) -> None:
        fr, pv = args
        check(lib().stitch_frame(self._h, fr, ctypes.byref(pv), stream_handle))

    def view(self, what: str, camera: int, level: int):
        """(tensor, (origin_x, origin_y)) aliasing the workspace; what in lap|gauss|mask|r."""
        code = {"lap": 0, "gauss": 1, "mask": 2, "r": 3}[what]
        im = StitchImage()
        ox, oy = c_int32(), c_int32()
        check(lib().stitch_plan_view(self._h, code, camera, level, ctypes.byref(im), ctypes.byref(ox),
                                     ctypes.byref(oy)))
        if im.width == 0 or im.height == 0:
            return None, (ox.value, oy.value)
        dt = _TORCH_DT[im.dtype]
        es = torch.empty((), dtype=dt).element_size()
        base = self.workspace.data_ptr()
        flat = self.workspace[: (self.workspace.numel() // es) * es].view(dt)
        off = im.data - base
        assert off % es == 0 and im.row_pitch % es == 0
        t = torch.as_strided(flat, (im.channels, im.height, im.width),
                             (im.plane_pitch // es if im.channels > 1 else 0, im.row_pitch // es, 1), off // es)
        return t, (ox.value, oy.value)

    def set_timing(self, enable: bool) -> None:
        check(lib().stitch_plan_set_timing(self._h, 1 if enable else 0))

    def read_timing(self) -> dict:
        """{kind: (total_ms, launches)} accumulated since set_timing(True)."""
        ms = (c_double * 8)()
        n = (c_int32 * 8)()
        check(lib().stitch_plan_read_timing(self._h, ms, n))
        return {TIMING_KINDS[i]: (ms[i], n[i]) for i in range(8) if n[i]}

    def config(self) -> dict:
        """{"wg_per_cu": [...], "tile_rows": [...]} of the plain form's pyramid passes."""
        wg = (c_int32 * MAX_LEVELS)()
        rows = (c_int32 * MAX_LEVELS)()
        check(lib().stitch_plan_config(self._h, wg, rows))
        return {"wg_per_cu": list(wg), "tile_rows": list(rows)}

    def set_config(self, wg_per_cu=None, tile_rows=None, stream=None) -> None:
        check(lib().stitch_plan_set_config(self._h, *_config_arrays(wg_per_cu, tile_rows), _stream(stream)))

    def autotune(self, frames, stream=None, cache_path=None) -> dict:
        """Time the pyramid passes' settings on these frames (stitch_autotune) and keep the
        fastest; returns config()."""
        fr = (StitchImage * self.n)(*[image_hwc(f) for f in frames])
        check(lib().stitch_autotune(self._h, fr, _stream(stream), str(cache_path).encode() if cache_path else None))
        return self.config()

    # ---- the plan as a differentiable function of float frames (stitch_frame_forward_f32,
    # ---- stitch_frame_backward); needs no bound workspace
    def _vjp_workspace(self, device):
        if getattr(self, "_vjp_ws", None) is None:
            nbytes = lib().stitch_frame_backward_workspace_bytes(self._h)
            if nbytes == 0:
                raise StitchError(2, "no workspace size for the differentiable form: " + last_error())
            self._vjp_ws = _aligned_workspace(nbytes, device) + (nbytes,)
        return self._vjp_ws

    def forward_f32(self, frames, stream=None) -> torch.Tensor:
        """R_0 (3, H, W) float32 of float (3, h, w) frames in [0, 1]."""
        frames = [f.contiguous() for f in frames]
        _, ws, nbytes = self._vjp_workspace(frames[0].device)
        r0 = torch.empty((3, self.canvas_h, self.canvas_w), dtype=torch.float32, device=frames[0].device)
        arr = (StitchImage * self.n)(*[image_chw(f) for f in frames])
        check(lib().stitch_frame_forward_f32(self._h, arr, ctypes.byref(image_chw(r0)), ws.data_ptr(), nbytes,
                                             _stream(stream)))
        return r0

    def backward(self, frames, d_pano, d_warped=None, stream=None):
        """(dl/dframes as n (3, h, w) float32 tensors, dl/dM as (n, 3, 3) float64) for the
        upstream dl/dR_0 d_pano (3, H, W) and optional direct terms d_warped[i] on the warped
        frames (None entries skipped)."""
        frames = [f.contiguous() for f in frames]
        dev = frames[0].device
        _, ws, nbytes = self._vjp_workspace(dev)
        outs = [torch.empty((3, h, w), dtype=torch.float32, device=dev) for w, h in self.frame_sizes]
        fa = (StitchImage * self.n)(*[image_chw(f) for f in frames])
        oa = (StitchImage * self.n)(*[image_chw(t) for t in outs])
        dp = d_pano.contiguous()
        keep = [dp]
        dw = None
        if d_warped is not None:
            views = []
            for t in d_warped:
                if t is None:
                    views.append(StitchImage())
                else:
                    t = t.contiguous()
                    keep.append(t)
                    views.append(image_chw(t))
            dw = (StitchImage * self.n)(*views)
        dh = (c_double * (9 * self.n))()
        check(lib().stitch_frame_backward(self._h, fa, ctypes.byref(image_chw(dp)), dw, oa, dh, ws.data_ptr(), nbytes,
                                          _stream(stream)))
        del keep
        return outs, np.array(dh[:], dtype=np.float64).reshape(self.n, 3, 3)

    def regions(self, camera: int, level: int):
        roi = (c_int32 * 4)()
        band = (c_int32 * 4)()
        check(lib().stitch_plan_regions(self._h, camera, level, roi, band))
        return tuple(roi), tuple(band)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().stitch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _config_arrays(wg_per_cu, tile_rows):
    wg = list(wg_per_cu or [])
    rows = list(tile_rows or [])
    return ((c_int32 * MAX_LEVELS)(*(wg + [0] * (MAX_LEVELS - len(wg)))),
            (c_int32 * MAX_LEVELS)(*(rows + [0] * (MAX_LEVELS - len(rows)))))


# ----------------------------------------------------------------------------- pipelined sequences
class Pipe:
    """Stream-pipelined frame sequences over a bound plan (Sec. 4.3.2, Fig. 3): host frame
    sets in, host panoramas out, with uploads, stitching and downloads on three streams."""

    def __init__(self, plan: "Plan", depth: int = 2):
        nbytes = lib().stitch_pipe_workspace_bytes(plan._h, depth)
        if nbytes == 0:
            raise StitchError(2, f"no pipe workspace for depth {depth}")
        self._buf, self._ws = _aligned_workspace(nbytes, plan.device)   # the device slots
        handle = c_void_p()
        check(lib().stitch_pipe_create(plan._h, depth, self._ws.data_ptr(), nbytes, ctypes.byref(handle)))
        self._h = handle
        self.plan = plan
        self.depth = depth

    def run(self, frames, panos) -> None:
        """frames: one list of n host uint8 (h, w, 3) tensors per frame set (pinned memory
        lets the copies overlap); panos: one host uint8 (H, W, 3) tensor per frame set.
        Returns when every panorama is on the host."""
        n = self.plan.n
        flat = [f for fs in frames for f in fs]
        if len(flat) != n * len(panos):
            raise ValueError("frames must hold n frames per panorama")
        for t in flat + list(panos):
            if t.device.type != "cpu" or t.dtype != torch.uint8 or not t.is_contiguous():
                raise ValueError("pipe frames and panoramas are contiguous host uint8 tensors")
        fp = (c_void_p * len(flat))(*[t.data_ptr() for t in flat])
        pp = (c_void_p * len(panos))(*[t.data_ptr() for t in panos])
        check(lib().stitch_pipe_run(self._h, len(panos), fp, pp))

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().stitch_pipe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many planned jobs per run: one launch per pyramid level and per blend level over
    every job's tiles, captured once into a HIP graph on a non-null stream."""

    def __init__(self, plans, device="cuda"):
        self.plans = list(plans)          # keeps the plans (and their workspaces) alive
        n = len(self.plans)
        arr = (c_void_p * n)(*[p._h for p in self.plans])
        h = c_void_p()
        check(lib().stitch_batch_create(n, arr, ctypes.byref(h)))
        self._h = h
        self.ws_bytes = lib().stitch_batch_workspace_bytes(self._h)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        base = (self.workspace.data_ptr() + 255) // 256 * 256
        check(lib().stitch_batch_bind(self._h, base, self.ws_bytes))
        self._args = None

    def _marshal(self, frames, panos):
        rows = [(StitchImage * len(f))(*[image_hwc(x) for x in f]) for f in frames]
        fr = (POINTER(StitchImage) * len(rows))(*[ctypes.cast(r, POINTER(StitchImage)) for r in rows])
        pv = (StitchImage * len(panos))(*[image_hwc(p) for p in panos])
        return rows, fr, pv

    def args(self, frames, panos):
        """Pre-marshalled arguments for repeated runs."""
        return self._marshal(frames, panos)

    def run(self, frames, panos, stream=None, args=None) -> None:
        a = args or self._marshal(frames, panos)
        check(lib().stitch_batch_run(self._h, a[1], a[2], _stream(stream)))

    def run_raw(self, args, stream_handle: int) -> None:
        check(lib().stitch_batch_run(self._h, args[1], args[2], stream_handle))

    def autotune(self, frames, panos, stream=None, cache_path=None):
        a = self._marshal(frames, panos)
        check(lib().stitch_batch_autotune(self._h, a[1], a[2], _stream(stream),
                                          None if cache_path is None else str(cache_path).encode()))
        return self.config()

    def set_timing(self, enable: bool) -> None:
        check(lib().stitch_batch_set_timing(self._h, 1 if enable else 0))

    def read_timing(self) -> dict:
        """{("pyr", k) or ("blend", k): (total_ms, launches)} accumulated since set_timing(True)."""
        ms = (c_double * (2 * MAX_LEVELS))()
        n = (c_int32 * (2 * MAX_LEVELS))()
        check(lib().stitch_batch_read_timing(self._h, ms, n))
        out = {}
        for i in range(2 * MAX_LEVELS):
            if n[i]:
                out[("pyr", i) if i < MAX_LEVELS else ("blend", i - MAX_LEVELS)] = (ms[i], n[i])
        return out

    def config(self) -> dict:
        """{"wg_per_cu": [...], "tile_rows": [...]} per pyramid level (tile_rows 0 past the
        last pass)."""
        wg = (c_int32 * MAX_LEVELS)()
        rows = (c_int32 * MAX_LEVELS)()
        check(lib().stitch_batch_config(self._h, wg, rows))
        return {"wg_per_cu": list(wg), "tile_rows": list(rows)}

    def set_config(self, wg_per_cu=None, tile_rows=None) -> None:
        """Per-pass settings (lists indexed by level; missing entries keep the tile height
        and take as many workgroups as fit)."""
        check(lib().stitch_batch_set_config(self._h, *_config_arrays(wg_per_cu, tile_rows)))

    def set_groups(self, groups: int) -> None:
        """Run the jobs as `groups` sub-batches pipelined over two streams (1: one sequence)."""
        check(lib().stitch_batch_set_groups(self._h, int(groups)))

    @property
    def groups(self) -> int:
        return lib().stitch_batch_group_count(self._h)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().stitch_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- differentiable pair form
def _dvec(a, n: int) -> ctypes.Array:
    a = np.asarray(a, dtype=np.float64).reshape(n)
    return (c_double * n)(*a.tolist())


def corners_to_h(q, w: int, h: int) -> np.ndarray:
    """H (3x3, h33 = 1) taking the corners of a w x h frame to the canvas points q (8,)."""
    out = (c_double * 9)()
    check(lib().stitch_corners_to_h(_dvec(q, 8), w, h, out))
    return np.array(out[:], dtype=np.float64).reshape(3, 3)


def map_grad_to_corners(q, w: int, h: int, d_map) -> np.ndarray:
    """d loss / d q (8,) from d loss / d M (3x3) of the frame whose corners sit at q."""
    out = (c_double * 8)()
    check(lib().stitch_map_grad_to_corners(_dvec(q, 8), w, h, _dvec(d_map, 9), out))
    return np.array(out[:], dtype=np.float64)


class Grad:
    """Loss of a stitched pair and its adjoint (float CHW frames in [0, 1]); cells and the
    overlap Omega are frozen by freeze().  One forward/backward in flight per object."""

    def __init__(self, frame_sizes, masks, canvas_w: int, canvas_h: int, levels: int, device="cuda"):
        self.frame_sizes = [tuple(map(int, s)) for s in frame_sizes]
        if len(self.frame_sizes) != 2 or len(masks) != 2:
            raise ValueError("the differentiable form takes a pair of frames")
        fw = (c_int32 * 2)(*[s[0] for s in self.frame_sizes])
        fh = (c_int32 * 2)(*[s[1] for s in self.frame_sizes])
        ms = [np.ascontiguousarray(np.asarray(m, dtype=np.uint8)) for m in masks]
        for m in ms:
            if m.shape != (canvas_h, canvas_w):
                raise ValueError("each mask must be (canvas_h, canvas_w) uint8")
        mptrs = (POINTER(c_uint8) * 2)(*[m.ctypes.data_as(POINTER(c_uint8)) for m in ms])
        h = c_void_p()
        check(lib().stitch_grad_create(fw, fh, mptrs, canvas_w, canvas_h, levels, ctypes.byref(h)))
        self._h = h
        self.masks, self.canvas_w, self.canvas_h, self.levels = ms, canvas_w, canvas_h, levels
        self.frozen_maps = None
        self._plan = None
        self.device = torch.device(device)
        self.ws_bytes = lib().stitch_grad_workspace_bytes(self._h)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = (self.workspace.data_ptr() + 255) // 256 * 256
        check(lib().stitch_grad_bind(self._h, base, self.ws_bytes, _stream(None)))
        self.omega = 0
        self._frames = None
        self.generation = 0

    @staticmethod
    def _h18(Hs) -> ctypes.Array:
        return _dvec(np.stack([np.asarray(H, dtype=np.float64).reshape(9) for H in Hs]), 18)

    def freeze(self, Hs, stream=None) -> int:
        n = c_int64()
        check(lib().stitch_grad_freeze(self._h, self._h18(Hs), ctypes.byref(n), _stream(stream)))
        self.omega = n.value
        self.frozen_maps = np.stack([np.asarray(H, dtype=np.float64) for H in Hs])
        return self.omega

    def upstream(self, stream=None):
        """The last forward's dl/dP and its direct terms dl/dA, dl/dB on the warped frames,
        as (3, H, W) float32 tensors (stitch_grad_upstream)."""
        outs = [torch.empty((3, self.canvas_h, self.canvas_w), dtype=torch.float32, device=self.device)
                for _ in range(3)]
        dw = (StitchImage * 2)(image_chw(outs[1]), image_chw(outs[2]))
        check(lib().stitch_grad_upstream(self._h, ctypes.byref(image_chw(outs[0])), dw, _stream(stream)))
        return outs[0], outs[1:]

    def plan_at(self, Hs) -> "Plan":
        """An unbound plan of the pair at the maps Hs (for stitch_frame_backward), reused
        while the maps stay the same."""
        key = np.stack([np.asarray(H, dtype=np.float64) for H in Hs])
        if self._plan is None or not np.array_equal(self._plan[0], key):
            self._plan = (key, Plan(self.frame_sizes, list(key), self.masks, self.canvas_w, self.canvas_h,
                                    self.levels, device=self.device, bind=False))
        return self._plan[1]

    def forward(self, frames, Hs, stream=None) -> float:
        frames = [f.contiguous() for f in frames]
        arr = (StitchImage * 2)(*[image_chw(f) for f in frames])
        loss = c_double()
        check(lib().stitch_grad_forward(self._h, arr, self._h18(Hs), ctypes.byref(loss), _stream(stream)))
        self._frames = frames          # the library reads them again in backward
        self.generation += 1
        return loss.value

    def backward(self, stream=None):
        """(d loss / d frames as two (3, h, w) float32 tensors, d loss / d M as (2, 3, 3))."""
        outs = [torch.empty((3, h, w), dtype=torch.float32, device=self.device) for w, h in self.frame_sizes]
        arr = (StitchImage * 2)(*[image_chw(t) for t in outs])
        dm = (c_double * 18)()
        check(lib().stitch_grad_backward(self._h, arr, dm, _stream(stream)))
        return outs, np.array(dm[:], dtype=np.float64).reshape(2, 3, 3)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().stitch_grad_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StitchPairLoss(torch.autograd.Function):
    """loss(frame_a, frame_b, q): camera A at the fixed homography H_a, camera B at the
    homography whose frame corners land on q (8 canvas coordinates, float64 CPU tensor).
    Gradients flow to both frames and to q."""

    @staticmethod
    def forward(ctx, frame_a, frame_b, q, grad: Grad, H_a):
        w, h = grad.frame_sizes[1]
        qn = q.detach().cpu().double().numpy().copy()
        H_b = corners_to_h(qn, w, h)
        maps = np.stack([np.asarray(H_a, dtype=np.float64), H_b])
        if grad.frozen_maps is None or not np.array_equal(grad.frozen_maps, maps):
            raise RuntimeError("freeze the Grad object at these maps first: the loss and its gradient take the "
                               "cells at the frozen maps")
        loss = grad.forward([frame_a.detach(), frame_b.detach()], [H_a, H_b])
        ctx.grad_obj, ctx.q, ctx.gen, ctx.maps = grad, qn, grad.generation, maps
        ctx.frames = (frame_a.detach(), frame_b.detach())
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g_out):
        grad = ctx.grad_obj
        if grad.generation != ctx.gen:
            raise RuntimeError("another forward ran on this Grad object since this loss was computed")
        # the loss's upstream gradients through the whole path's vector-Jacobian product
        d_pano, d_warped = grad.upstream()
        d_frames, d_map = grad.plan_at(ctx.maps).backward(list(ctx.frames), d_pano, d_warped)
        w, h = grad.frame_sizes[1]
        dq = torch.from_numpy(map_grad_to_corners(ctx.q, w, h, d_map[1]))
        gs = float(g_out)
        return d_frames[0] * gs, d_frames[1] * gs, dq * gs, None, None


def refine_pair(grad: Grad, frame_a, frame_b, H_a, q0, steps: int = 50, lr: float = 1e-3,
                record=(0, 10, 25, 50), q_true=None):
    """Adam (betas 0.9/0.999, eps 1e-8) on the normalised corners q~ = (q_x / (w/2),
    q_y / (h/2)) of frame B.  Before every step the cells and Omega are frozen at the
    current corners, so each gradient is the exact one of the loss piece the corners are
    on.  Returns (q, {step: (loss, mean corner distance to q_true in px, or None)})."""
    w, h = grad.frame_sizes[1]
    scale = torch.tensor([w / 2.0, h / 2.0] * 4, dtype=torch.float64)
    qt = (torch.as_tensor(np.asarray(q0, dtype=np.float64)) / scale).requires_grad_(True)
    opt = torch.optim.Adam([qt], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    log = {}

    def err(qv):
        if q_true is None:
            return None
        d = (qv - np.asarray(q_true, dtype=np.float64)).reshape(4, 2)
        return float(np.mean(np.linalg.norm(d, axis=1)))

    for step in range(steps + 1):
        q = (qt * scale)
        qn = q.detach().numpy()
        grad.freeze([H_a, corners_to_h(qn, w, h)])
        opt.zero_grad()
        loss = StitchPairLoss.apply(frame_a, frame_b, q, grad, H_a)
        if step in record:
            log[step] = (float(loss), err(qn))
        if step == steps:
            break
        loss.backward()
        opt.step()
    return (qt * scale).detach().numpy(), log


# ----------------------------------------------------------------------------- L-ORB features
def detection_areas(frame_sizes, Hs, canvas_w: int, canvas_h: int, margin: int = 24) -> list:
    """Per camera, the feature detection areas (x, y, w, h) of its frame (Alg. 2, step 1):
    where the footprints of the pre-aligned neighbours overlap it, by stitch_detection_areas
    (host-only)."""
    n = len(frame_sizes)
    fw = (c_int32 * n)(*[int(w) for w, _ in frame_sizes])
    fh = (c_int32 * n)(*[int(h) for _, h in frame_sizes])
    hs = (c_double * (9 * n))(*[float(v) for H in Hs for v in np.asarray(H, dtype=np.float64).reshape(9)])
    cap = max(1, n - 1)
    counts = (c_int32 * n)()
    out = (c_int32 * (4 * n * cap))()
    check(lib().stitch_detection_areas(n, fw, fh, hs, int(canvas_w), int(canvas_h), int(margin), cap, counts, out))
    return [[tuple(out[4 * (k * cap + a) + i] for i in range(4)) for a in range(counts[k])] for k in range(n)]


class Lorb:
    """L-ORB feature extraction (Sec. 4.1, Alg. 1 and Alg. 2) in fixed detection areas of
    frames of one size: device outputs and workspace are allocated once and reused."""

    def __init__(self, frame_w: int, frame_h: int, areas, n_max: int = 500, nd: int = 256,
                 fast_threshold: int = 20, harris_threshold: int = 0, device="cuda"):
        self.frame_w, self.frame_h = int(frame_w), int(frame_h)
        flat = [int(v) for r in areas for v in r]
        self.m = len(flat) // 4
        self.areas = (c_int32 * max(len(flat), 1))(*flat)
        self.n_max, self.nd = int(n_max), int(nd)
        self.tf, self.t = int(fast_threshold), int(harris_threshold)
        nbytes = lib().stitch_lorb_workspace_bytes(self.frame_w, self.frame_h, self.m, self.areas)
        if nbytes == 0:
            raise StitchError(2, "no workspace size for these areas")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        m, n, words = self.m, self.n_max, 2 * self.nd // 32
        self.counts = torch.zeros(m, dtype=torch.int32, device=device)
        self.points = torch.zeros(m, n, 2, dtype=torch.int32, device=device)
        self.responses = torch.zeros(m, n, dtype=torch.int64, device=device)
        self.descriptors = torch.zeros(m, n, words, dtype=torch.int32, device=device)

    def run_raw(self, frame: torch.Tensor, pattern: torch.Tensor, stream_handle: int) -> None:
        """Queue the extraction of `frame` (H, W, 3 uint8 device) with `pattern` (nd, 4 int32
        device) on a raw stream handle; outputs land in counts/points/responses/descriptors."""
        img = image_hwc(frame)
        _on_gpu(pattern, "pattern")
        check(lib().stitch_lorb(ctypes.byref(img), self.m, self.areas, self.tf, self.t, self.n_max, self.nd,
                                pattern.data_ptr(), self.counts.data_ptr(), self.points.data_ptr(),
                                self.responses.data_ptr(), self.descriptors.data_ptr(), self._ws.data_ptr(),
                                self._ws.numel(), stream_handle))

    def run(self, frame: torch.Tensor, pattern: torch.Tensor, stream=None) -> list:
        """Extract and return, per area, (points (k, 2) int32, responses (k,) int64,
        descriptors (k, 2 nd/32) uint32 as int32 bits), k = that area's count."""
        if pattern.dtype != torch.int32 or tuple(pattern.shape) != (self.nd, 4) or not pattern.is_contiguous():
            raise ValueError(f"pattern must be a contiguous ({self.nd}, 4) int32 tensor")
        if frame.dtype != torch.uint8 or frame.dim() != 3 or frame.shape[2] != 3:
            raise ValueError("frame must be an (H, W, 3) uint8 tensor")
        if frame.shape[0] != self.frame_h or frame.shape[1] != self.frame_w:
            raise ValueError("frame size differs from the one the areas were sized for")
        self.run_raw(frame, pattern, _stream(stream))
        torch.cuda.synchronize()
        counts = self.counts.cpu().tolist()
        return [(self.points[i, :k].cpu(), self.responses[i, :k].cpu(), self.descriptors[i, :k].cpu())
                for i, k in enumerate(counts)]


class LorbSet:
    """L-ORB in the areas of several frames with one call (stitch_lorb_multi): frame_sizes
    [(w, h)] and areas_per_frame [[(x, y, w, h), ...], ...]; outputs indexed by the areas in
    frame order."""

    def __init__(self, frame_sizes, areas_per_frame, n_max: int = 500, nd: int = 256, fast_threshold: int = 20,
                 harris_threshold: int = 0, device="cuda"):
        self.nframes = len(frame_sizes)
        self.fw = (c_int32 * self.nframes)(*[int(w) for w, _ in frame_sizes])
        self.fh = (c_int32 * self.nframes)(*[int(h) for _, h in frame_sizes])
        self.mpf = (c_int32 * self.nframes)(*[len(a) for a in areas_per_frame])
        flat = [int(v) for a in areas_per_frame for r in a for v in r]
        self.m = len(flat) // 4
        self.areas = (c_int32 * max(len(flat), 1))(*flat)
        self.n_max, self.nd = int(n_max), int(nd)
        self.tf, self.t = int(fast_threshold), int(harris_threshold)
        nbytes = lib().stitch_lorb_multi_workspace_bytes(self.nframes, self.fw, self.fh, self.mpf, self.areas)
        if nbytes == 0:
            raise StitchError(2, "no workspace size for these areas: " + last_error())
        self._buf, self._ws = _aligned_workspace(nbytes, device)
        m, n, words = self.m, self.n_max, 2 * self.nd // 32
        self.counts = torch.zeros(m, dtype=torch.int32, device=device)
        self.points = torch.zeros(m, n, 2, dtype=torch.int32, device=device)
        self.responses = torch.zeros(m, n, dtype=torch.int64, device=device)
        self.descriptors = torch.zeros(m, n, words, dtype=torch.int32, device=device)

    def run_raw(self, frames, pattern: torch.Tensor, stream_handle: int) -> None:
        imgs = (StitchImage * self.nframes)(*[image_hwc(f) for f in frames])
        _on_gpu(pattern, "pattern")
        check(lib().stitch_lorb_multi(self.nframes, imgs, self.mpf, self.areas, self.tf, self.t, self.n_max, self.nd,
                                      pattern.data_ptr(), self.counts.data_ptr(), self.points.data_ptr(),
                                      self.responses.data_ptr(), self.descriptors.data_ptr(), self._ws.data_ptr(),
                                      self._ws.numel(), stream_handle))


LORB_KINDS = ["clear", "detect", "select", "rank", "brief"]


def lorb_set_timing(enable: bool) -> None:
    """Per-launch event timing of every stitch_lorb call in the process (clears totals)."""
    check(lib().stitch_lorb_set_timing(int(enable)))


def lorb_read_timing() -> dict:
    """{launch: (total ms, launches)} over the calls since lorb_set_timing."""
    ms = (c_double * len(LORB_KINDS))()
    n = (c_int32 * len(LORB_KINDS))()
    check(lib().stitch_lorb_read_timing(ms, n))
    return {k: (ms[i], n[i]) for i, k in enumerate(LORB_KINDS)}


# ----------------------------------------------------------------------------- registration
def _aligned_workspace(nbytes: int, device) -> tuple:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf[off:off + nbytes]


class Matcher:
    """Multi-probe LSH matching (Sec. 4.2.1; Alg. 3, step 1) of two descriptor sets with
    capacities cap_a, cap_b: positions is a (tables, kbits) int array of gt-bit indices."""

    def __init__(self, cap_a: int, cap_b: int, nd: int, positions, max_dist: int, device="cuda"):
        pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int32).reshape(len(positions), -1))
        self.tables, self.kbits = pos.shape
        self.positions = (c_int32 * max(pos.size, 1))(*pos.reshape(-1).tolist())
        self.cap_a, self.cap_b, self.nd, self.max_dist = int(cap_a), int(cap_b), int(nd), int(max_dist)
        nbytes = lib().stitch_lsh_match_workspace_bytes(self.cap_a, self.cap_b, self.tables)
        if nbytes == 0:
            raise StitchError(2, "no workspace size for these capacities")
        self._buf, self._ws = _aligned_workspace(nbytes, device)
        self.match = torch.full((self.cap_a,), -1, dtype=torch.int32, device=device)
        self.dist = torch.full((self.cap_a,), -1, dtype=torch.int32, device=device)

    def run_raw(self, desc_a, count_a, desc_b, count_b, stream_handle: int) -> None:
        for t, name in ((desc_a, "desc_a"), (count_a, "count_a"), (desc_b, "desc_b"), (count_b, "count_b")):
            _on_gpu(t, name)
        check(lib().stitch_lsh_match(self.nd, desc_a.data_ptr(), count_a.data_ptr(), self.cap_a, desc_b.data_ptr(),
                                     count_b.data_ptr(), self.cap_b, self.tables, self.kbits, self.positions,
                                     self.max_dist, self.match.data_ptr(), self.dist.data_ptr(),
                                     self._ws.data_ptr(), self._ws.numel(), stream_handle))

    def run(self, desc_a, count_a, desc_b, count_b, stream=None):
        """desc_*: (cap, 2 nd/32) int32/uint32 device tensors, count_*: one-element int32
        device tensors.  Returns (match, dist) as host tensors."""
        for d, cap in ((desc_a, self.cap_a), (desc_b, self.cap_b)):
            if d.dtype != torch.int32 or d.dim() != 2 or d.shape[0] < cap or d.shape[1] != 2 * self.nd // 32 \
                    or not d.is_contiguous() or not d.is_cuda:
                raise ValueError("descriptors must be contiguous int32 device tensors of (cap, 2 nd/32)")
        for c in (count_a, count_b):
            if c.dtype != torch.int32 or not c.is_cuda or c.numel() < 1:
                raise ValueError("counts must be int32 device tensors")
        self.run_raw(desc_a, count_a, desc_b, count_b, _stream(stream))
        torch.cuda.synchronize()
        return self.match.cpu(), self.dist.cpu()


class Prosac:
    """PROSAC (Sec. 4.2.2; Alg. 3, step 2; Alg. 4, step 5) over the matches of one pair,
    with nhyp hypotheses drawn from caller-supplied uniforms."""

    def __init__(self, cap_a: int, cap_b: int, nhyp: int, T_N: float = 200000.0, eps: float = 3.0,
                 device="cuda"):
        self.cap_a, self.cap_b, self.nhyp = int(cap_a), int(cap_b), int(nhyp)
        self.T_N, self.eps = float(T_N), float(eps)
        nbytes = lib().stitch_prosac_workspace_bytes(self.cap_a, self.nhyp)
        if nbytes == 0:
            raise StitchError(2, "no workspace size for these capacities")
        self._buf, self._ws = _aligned_workspace(nbytes, device)
        self.H = torch.zeros(9, dtype=torch.float64, device=device)
        self.inliers = torch.zeros(1, dtype=torch.int32, device=device)
        self.mask = torch.zeros(self.cap_a, dtype=torch.uint8, device=device)
        self.hyp_counts = torch.zeros(self.nhyp, dtype=torch.int32, device=device)

    def run_raw(self, pts_a, pts_b, match, dist, count_a, uniforms, stream_handle: int) -> None:
        for t, name in ((pts_a, "pts_a"), (pts_b, "pts_b"), (match, "match"), (dist, "dist"), (count_a, "count_a"),
                        (uniforms, "uniforms")):
            _on_gpu(t, name)
        check(lib().stitch_prosac(pts_a.data_ptr(), pts_b.data_ptr(), self.cap_b, match.data_ptr(), dist.data_ptr(),
                                  count_a.data_ptr(), self.cap_a, self.nhyp, uniforms.data_ptr(), self.T_N, self.eps,
                                  self.H.data_ptr(), self.inliers.data_ptr(), self.mask.data_ptr(),
                                  self.hyp_counts.data_ptr(), self._ws.data_ptr(), self._ws.numel(),
                                  stream_handle))

    def run(self, pts_a, pts_b, match, dist, count_a, uniforms, stream=None) -> dict:
        """pts_*: (cap, 2) int32 device, match/dist: (cap_a,) int32 device, count_a: one-element
        int32 device, uniforms: (nhyp, 4) float64 device in [0, 1)."""
        if uniforms.dtype != torch.float64 or tuple(uniforms.shape) != (self.nhyp, 4) or not uniforms.is_contiguous():
            raise ValueError(f"uniforms must be a contiguous ({self.nhyp}, 4) float64 tensor")
        for t, n, name in ((pts_a, 2 * self.cap_a, "pts_a"), (pts_b, 2 * self.cap_b, "pts_b"),
                           (match, self.cap_a, "match"), (dist, self.cap_a, "dist"), (count_a, 1, "count_a")):
            if t.dtype != torch.int32 or not t.is_contiguous() or t.numel() < n or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous int32 device tensor of at least {n} elements")
        self.run_raw(pts_a, pts_b, match, dist, count_a, uniforms, _stream(stream))
        torch.cuda.synchronize()
        return {"H": self.H.cpu().numpy().reshape(3, 3), "inliers": int(self.inliers[0]),
                "mask": self.mask.cpu().numpy().astype(bool), "hyp_counts": self.hyp_counts.cpu().numpy()}


class MatcherSet:
    """Matching (Sec. 4.2.1; Alg. 3, step 1) of several area pairs with one launch per stage
    (stitch_lsh_match_multi): caps is [(cap_a, cap_b)] per pair, the settings are shared.
    Pair p's outputs match[p], dist[p] (cap_a entries) equal a Matcher's for that pair."""

    def __init__(self, caps, nd: int, positions, max_dist: int, device="cuda"):
        pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int32).reshape(len(positions), -1))
        self.tables, self.kbits = pos.shape
        self.positions = (c_int32 * max(pos.size, 1))(*pos.reshape(-1).tolist())
        self.caps = [(int(a), int(b)) for a, b in caps]
        self.n, self.nd, self.max_dist = len(self.caps), int(nd), int(max_dist)
        self.pairs = (MatchPair * max(self.n, 1))()
        for p, (a, b) in enumerate(self.caps):
            self.pairs[p].cap_a, self.pairs[p].cap_b = a, b
        nbytes = lib().stitch_lsh_match_multi_workspace_bytes(self.n, self.pairs, self.tables)
        if nbytes == 0:
            raise StitchError(2, "no workspace size for these pairs and tables")
        self._buf, self._ws = _aligned_workspace(nbytes, device)
        self.match = [torch.full((a,), -1, dtype=torch.int32, device=device) for a, _ in self.caps]
        self.dist = [torch.full((a,), -1, dtype=torch.int32, device=device) for a, _ in self.caps]

    def run_raw(self, inputs, stream_handle: int) -> None:
        """inputs: per pair (desc_a, count_a, desc_b, count_b) device tensors."""
        if len(inputs) != self.n:
            raise ValueError(f"{len(inputs)} input pairs for a set of {self.n}")
        for p, (da, ca, db, cb) in enumerate(inputs):
            for t, name in ((da, "desc_a"), (ca, "count_a"), (db, "desc_b"), (cb, "count_b")):
                _on_gpu(t, f"pair {p} {name}")
            e = self.pairs[p]
            e.desc_a, e.count_a, e.desc_b, e.count_b = da.data_ptr(), ca.data_ptr(), db.data_ptr(), cb.data_ptr()
            e.match, e.dist = self.match[p].data_ptr(), self.dist[p].data_ptr()
        check(lib().stitch_lsh_match_multi(self.n, self.pairs, self.nd, self.tables, self.kbits, self.positions,
                                           self.max_dist, self._ws.data_ptr(), self._ws.numel(), stream_handle))

    def run(self, inputs, stream=None):
        """inputs: per pair (desc_a, count_a, desc_b, count_b) as for Matcher.run.  Returns
        [(match, dist)] as host tensors."""
        if len(inputs) != self.n:
            raise ValueError(f"{len(inputs)} input pairs for a set of {self.n}")
        for (da, ca, db, cb), (cap_a, cap_b) in zip(inputs, self.caps):
            for d, cap in ((da, cap_a), (db, cap_b)):
                if d.dtype != torch.int32 or d.dim() != 2 or d.shape[0] < cap or d.shape[1] != 2 * self.nd // 32 \
                        or not d.is_contiguous() or not d.is_cuda:
                    raise ValueError("descriptors must be contiguous int32 device tensors of (cap, 2 nd/32)")
            for c in (ca, cb):
                if c.dtype != torch.int32 or not c.is_cuda or c.numel() < 1:
                    raise ValueError("counts must be int32 device tensors")
        self.run_raw(inputs, _stream(stream))
        torch.cuda.synchronize()
        return [(m.cpu(), d.cpu()) for m, d in zip(self.match, self.dist)]


class ProsacSet:
    """PROSAC (Sec. 4.2.2; Alg. 3, step 2) of several area pairs with one launch per stage
    (stitch_prosac_multi), nhyp hypotheses each; caps is [(cap_a, cap_b)] per pair.  Pair
    p's H[p] (9 float64), inliers[p], mask[p] (cap_a) and hyp_counts[p] equal a Prosac's."""

    def __init__(self, caps, nhyp: int, T_N: float = 200000.0, eps: float = 3.0, device="cuda"):
        self.caps = [(int(a), int(b)) for a, b in caps]
        self.n, self.nhyp = len(self.caps), int(nhyp)
        self.T_N, self.eps = float(T_N), float(eps)
        self.pairs = (ProsacPair * max(self.n, 1))()
        for p, (a, b) in enumerate(self.caps):
            self.pairs[p].cap_a, self.pairs[p].cap_b = a, b
        nbytes = lib().stitch_prosac_multi_workspace_bytes(self.n, self.pairs, self.nhyp)
        if nbytes == 0:
            raise StitchError(2, "no workspace size for these pairs and hypotheses")
        self._buf, self._ws = _aligned_workspace(nbytes, device)
        self.H = torch.zeros(max(self.n, 1), 9, dtype=torch.float64, device=device)
        self.inliers = torch.zeros(max(self.n, 1), dtype=torch.int32, device=device)
        self.mask = [torch.zeros(a, dtype=torch.uint8, device=device) for a, _ in self.caps]
        self.hyp_counts = torch.zeros(max(self.n, 1), self.nhyp, dtype=torch.int32, device=device)

    def run_raw(self, inputs, stream_handle: int) -> None:
        """inputs: per pair (pts_a, pts_b, match, dist, count_a, uniforms) device tensors."""
        if len(inputs) != self.n:
            raise ValueError(f"{len(inputs)} input pairs for a set of {self.n}")
        for p, (pa, pb, m, d, ca, u) in enumerate(inputs):
            for t, name in ((pa, "pts_a"), (pb, "pts_b"), (m, "match"), (d, "dist"), (ca, "count_a"),
                            (u, "uniforms")):
                _on_gpu(t, f"pair {p} {name}")
            e = self.pairs[p]
            e.pts_a, e.pts_b, e.match, e.dist = pa.data_ptr(), pb.data_ptr(), m.data_ptr(), d.data_ptr()
            e.count_a, e.uniforms = ca.data_ptr(), u.data_ptr()
            e.H, e.inliers = self.H[p].data_ptr(), self.inliers[p:p + 1].data_ptr()
            e.inlier_mask, e.hyp_counts = self.mask[p].data_ptr(), self.hyp_counts[p].data_ptr()
        check(lib().stitch_prosac_multi(self.n, self.pairs, self.nhyp, self.T_N, self.eps, self._ws.data_ptr(),
                                        self._ws.numel(), stream_handle))

    def run(self, inputs, stream=None) -> list:
        """inputs: per pair (pts_a, pts_b, match, dist, count_a, uniforms) as for Prosac.run.
        Returns one dict per pair (H, inliers, mask, hyp_counts) on the host."""
        if len(inputs) != self.n:
            raise ValueError(f"{len(inputs)} input pairs for a set of {self.n}")
        for (pa, pb, m, d, ca, u), (cap_a, cap_b) in zip(inputs, self.caps):
            if u.dtype != torch.float64 or tuple(u.shape) != (self.nhyp, 4) or not u.is_contiguous():
                raise ValueError(f"uniforms must be a contiguous ({self.nhyp}, 4) float64 tensor")
            for t, n, name in ((pa, 2 * cap_a, "pts_a"), (pb, 2 * cap_b, "pts_b"), (m, cap_a, "match"),
                               (d, cap_a, "dist"), (ca, 1, "count_a")):
                if t.dtype != torch.int32 or not t.is_contiguous() or t.numel() < n or not t.is_cuda:
                    raise ValueError(f"{name} must be a contiguous int32 device tensor of at least {n} elements")
        self.run_raw(inputs, _stream(stream))
        torch.cuda.synchronize()
        return [{"H": self.H[p].cpu().numpy().reshape(3, 3), "inliers": int(self.inliers[p]),
                 "mask": self.mask[p].cpu().numpy().astype(bool), "hyp_counts": self.hyp_counts[p].cpu().numpy()}
                for p in range(self.n)]
