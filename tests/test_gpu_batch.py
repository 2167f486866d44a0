"""The batched form: many heterogeneous jobs per run, one launch per level over all
jobs, captured into a HIP graph.  Its output must equal the jobs stitched one by one,
bit for bit, on every replay; one job is also checked against the oracle directly."""
import numpy as np
import pytest
import torch

import oracle as o
import paper_1810_03988_amd as P
import workloads as wl
from helpers import assert_u8_parity, gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]
DEV = "cuda"
SMALL = [(160, 120), (320, 180), (256, 144), (480, 270)]


def _jobs(njobs=7, storage="f32"):
    rigs = wl.rig_c3_jobs(njobs, resolutions=SMALL)
    plans, frames, panos = [], [], []
    for r in rigs:
        assert r.levels >= 2
        plans.append(P.Plan(r.frame_sizes, r.H, r.masks(), r.canvas_w, r.canvas_h, r.levels, storage=storage))
        frames.append([f.to(DEV) for f in wl.render_rig_frames(r)])
        panos.append(torch.empty((r.canvas_h, r.canvas_w, 3), dtype=torch.uint8, device=DEV))
    return rigs, plans, frames, panos


def _one_by_one(plans, frames):
    return [p.frame(f).clone() for p, f in zip(plans, frames)]


def test_batched_graph_equals_one_by_one_on_every_replay():
    rigs, plans, frames, panos = _jobs()
    ref = _one_by_one(plans, frames)
    torch.cuda.synchronize()
    b = P.Batch(plans)
    s = torch.cuda.Stream()
    for rep in range(3):
        for p in panos:
            p.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.run(frames, panos, stream=s)
        s.synchronize()
        # eager work and a sync between replays
        _ = torch.ones(1000, device=DEV).sum().item()
        for j, (a, c) in enumerate(zip(panos, ref)):
            assert torch.equal(a, c), f"replay {rep}, job {j}"


def test_batched_follows_new_frames_and_null_stream():
    rigs, plans, frames, panos = _jobs(5)
    b = P.Batch(plans)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.run(frames, panos, stream=s)
    s.synchronize()
    # new frame buffers with other content: the tables follow, the graph is replayed
    frames2 = [[torch.flip(f, dims=[1]).contiguous() for f in fr] for fr in frames]
    ref2 = _one_by_one(plans, frames2)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        b.run(frames2, panos, stream=s)
    s.synchronize()
    for a, c in zip(panos, ref2):
        assert torch.equal(a, c)
    # the null stream takes the eager path
    for p in panos:
        p.zero_()
    b.run(frames, panos, stream=0)
    torch.cuda.synchronize()
    for a, c in zip(panos, _one_by_one(plans, frames)):
        assert torch.equal(a, c)


def test_batched_job_matches_the_oracle():
    rigs, plans, frames, panos = _jobs(4)
    b = P.Batch(plans)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.run(frames, panos, stream=s)
    s.synchronize()
    j = min(range(len(rigs)), key=lambda i: rigs[i].canvas_pixels())
    r = rigs[j]
    want = o.StitchOracle([f.cpu().numpy() for f in frames[j]], r.H, r.masks(), r.canvas_w, r.canvas_h,
                          r.levels).panorama()
    assert_u8_parity(panos[j].cpu().numpy(), want)


def test_autotune_keeps_results_and_uses_its_cache(tmp_path):
    rigs, plans, frames, panos = _jobs(4)
    ref = _one_by_one(plans, frames)
    b = P.Batch(plans)
    s = torch.cuda.Stream()
    cache = tmp_path / "tune.txt"
    with torch.cuda.stream(s):
        cfg = b.autotune(frames, panos, stream=s, cache_path=cache)
    assert cache.exists() and len(cache.read_text().strip().splitlines()) == 1
    nl = max(r.levels for r in rigs) - 1
    assert all(c in (0, 1, 2, -1) for c in cfg["wg_per_cu"])
    assert all(t in (16, 32, 64, 128) for t in cfg["tile_rows"][:nl]) and not any(cfg["tile_rows"][nl:])
    b2 = P.Batch(plans)
    with torch.cuda.stream(s):
        cfg2 = b2.autotune(frames, panos, stream=s, cache_path=cache)
        b2.run(frames, panos, stream=s)
    s.synchronize()
    assert cfg2 == cfg and len(cache.read_text().strip().splitlines()) == 1
    for a, c in zip(panos, ref):
        assert torch.equal(a, c)


@pytest.mark.parametrize("groups", [2, 3, 7])
def test_grouped_schedule_equals_one_by_one(groups):
    """The jobs as sub-batches pipelined over two streams: every replay equals one by one,
    also after new frame buffers and after the settings change."""
    rigs, plans, frames, panos = _jobs()
    ref = _one_by_one(plans, frames)
    torch.cuda.synchronize()
    b = P.Batch(plans)
    b.set_groups(groups)
    assert b.groups == groups
    s = torch.cuda.Stream()
    for rep in range(3):
        for p in panos:
            p.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.run(frames, panos, stream=s)
        s.synchronize()
        _ = torch.ones(1000, device=DEV).sum().item()
        for j, (a, c) in enumerate(zip(panos, ref)):
            assert torch.equal(a, c), f"replay {rep}, job {j}"
    b.set_config([-1] * 8, [32] * 8)
    frames2 = [[torch.flip(f, dims=[0]).contiguous() for f in fr] for fr in frames]
    ref2 = _one_by_one(plans, frames2)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        b.run(frames2, panos, stream=s)
    s.synchronize()
    for a, c in zip(panos, ref2):
        assert torch.equal(a, c)
