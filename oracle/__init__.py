"""Test infrastructure: a plain, slow FP64 CPU oracle of the per-frame stitching path.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import it.
The product path (paper_1810_03988_amd) never imports, links or calls anything here.
"""
from .stitch_oracle import (  # noqa: F401
    W5, reflect101, level_dims, hinv_spec, hinv_ideal, warp, warp_coords, reduce_at, expand_at,
    reduce_full, expand_full, gaussian_pyramid, laplacian_pyramid, collapse, quantise,
    blend_pyramids, StitchOracle, check_masks,
)
from .adjoint_oracle import (  # noqa: F401
    GradOracle, FrameVjpOracle, dlt_from_corners, dlt_jacobian, canvas_map_jacobian, reduce_T, expand_T,
    corners,
)
from .areas_oracle import detection_areas, footprint  # noqa: F401
