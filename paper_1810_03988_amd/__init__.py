"""MI355X-native per-frame panorama stitching path (warp + multi-band blend).

The compute runs in hand-written gfx950 HIP kernels behind the C ABI declared in
include/stitch.h (libstitch.so, built in-tree by paper_1810_03988_amd.build);
paper_1810_03988_amd.stitch is the ctypes binding.
"""
from . import stitch  # noqa: F401
from .stitch import (Batch, Grad, Lorb, LorbSet, Matcher, MatcherSet, Pipe, Plan, Prosac, ProsacSet,  # noqa: F401
                     StitchError, StitchPairLoss, blend, corners_to_h, detection_areas, lib,
                     map_grad_to_corners, pyramid, refine_pair, warp, warp_coords)
