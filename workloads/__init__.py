"""Seeded synthetic camera rigs and frames shaped like the paper's panoramic workloads.

This package builds inputs only (frames, source->canvas homographies, seam masks).
It holds none of the stitching arithmetic, so the HIP path and the oracle can both
consume it without sharing any of the method.
"""
from .synth import (  # noqa: F401
    ROOT_SEED, Rig, rig_c1, rig_c2, rig_c4, rig_c3_jobs, rig_c5_pairs, rig_ring,
    render_frames, render_rig_frames, render_rig_sequence, seam_masks, hash32_noise, scene_params,
    brief_pattern, rotated_frame,
)
