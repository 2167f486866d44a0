"""The stream-pipelined sequence form (host frame sets in, host panoramas out, uploads,
stitching and downloads on three streams) against stitch_frame one frame set at a time."""
import pytest
import torch

import paper_1810_03988_amd as P
import workloads as wl
from helpers import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _sequence(rig, count):
    return wl.render_rig_sequence(rig, range(count))


@pytest.mark.parametrize("depth, pinned", [(1, True), (2, True), (3, True), (2, False)])
def test_pipelined_sequence_equals_one_frame_set_at_a_time(depth, pinned):
    """Seven frame sets through depths 1-3 (slots reused several times), pinned and pageable
    host memory: every panorama equals the one stitch_frame gives bit for bit."""
    rig = wl.rig_c1()
    seq = _sequence(rig, 7)
    plan = P.Plan(rig.frame_sizes, rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels)
    want = [plan.frame([f.cuda() for f in fs]).cpu() for fs in seq]
    torch.cuda.synchronize()
    host = [[f.pin_memory() if pinned else f.clone() for f in fs] for fs in seq]
    panos = [torch.full((rig.canvas_h, rig.canvas_w, 3), 7, dtype=torch.uint8, pin_memory=pinned) for _ in seq]
    pipe = P.Pipe(plan, depth)
    pipe.run(host, panos)
    for t, (got, ref) in enumerate(zip(panos, want)):
        assert torch.equal(got, ref), f"frame set {t}"
    # a second run on the same pipe (slots and events reused) and an empty run
    panos2 = [torch.zeros_like(p) for p in panos[:3]]
    pipe.run(host[:3], panos2)
    pipe.run([], [])
    for got, ref in zip(panos2, want[:3]):
        assert torch.equal(got, ref)
    pipe.close()


def test_pipelined_panoramas_match_the_oracle():
    """Two frame sets of the two-camera rig through a depth-2 pipe (the second set has its
    own noise), each panorama against the FP64 oracle on the whole canvas: no sample off by
    more than 1, at most 0.01 % of the 3 x 1040 x 480 x 2 samples off by one."""
    import numpy as np
    import oracle as o
    from helpers import assert_u8_parity
    rig = wl.rig_c1()
    seq = _sequence(rig, 2)
    plan = P.Plan(rig.frame_sizes, rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels)
    host = [[f.pin_memory() for f in fs] for fs in seq]
    panos = [torch.zeros((rig.canvas_h, rig.canvas_w, 3), dtype=torch.uint8, pin_memory=True) for _ in seq]
    pipe = P.Pipe(plan, 2)
    pipe.run(host, panos)
    pipe.close()
    got, want = [], []
    for fs, pano in zip(seq, panos):
        so = o.StitchOracle([f.numpy() for f in fs], rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels)
        got.append(pano.numpy().reshape(-1))
        want.append(so.panorama().reshape(-1))
    assert not np.array_equal(want[0], want[1])
    assert_u8_parity(np.concatenate(got), np.concatenate(want), max_frac=1e-4)
