"""The batched form (many jobs, one launch per level over all of them; Sec. 4.3.2's images
of different sizes in flight) at the sizes and in the launch settings the benchmark runs:
jobs from the heterogeneous batching workload (one 3840x2160 four-camera job at 7 levels,
1920x1080 at 6, 1280x720 at 5, 640x480 at 4), tiles of 16 to 128 rows, persistent or
one-workgroup-per-tile grids, FP32 and FP16 storage.  The batched panoramas must equal
the jobs stitched one by one bit for bit in every setting, and the FP64 oracle checks
R_0, the bands and the uint8 output on windows through their dependency cones."""
import numpy as np
import pytest
import torch

import oracle as o
import paper_1810_03988_amd as P
import workloads as wl
from helpers import assert_float_parity, assert_u8_parity, gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]
DEV = "cuda"
SUBSET = (2, 3, 7, 13)          # jobs of the 64-job draw: 4K/L7, 1080p/L6, 720p/L5, 480p/L4
U16 = 2.0 ** -11


def _fp16_r0_bound(L):
    """Worst-case FP16 storage error of R_0 (derivation in test_gpu_precision)."""
    eB = [(2 * k + 1) * U16 + 2 * k * U16 for k in range(L)]
    eB[L - 1] = (L - 1) * U16 + 2 * (L - 1) * U16
    return sum(eB[j] + U16 for j in range(L))


def _setup(storage):
    rigs = [wl.rig_c3_jobs(max(SUBSET) + 1)[j] for j in SUBSET]
    assert [r.levels for r in rigs] == [7, 6, 5, 4] and rigs[0].frame_sizes[0] == (3840, 2160)
    plans = [P.Plan(r.frame_sizes, r.H, r.masks(), r.canvas_w, r.canvas_h, r.levels, storage=storage, keep_r0=True)
             for r in rigs]
    frames = [wl.render_rig_frames(r, 0, DEV) for r in rigs]
    panos = [torch.empty((r.canvas_h, r.canvas_w, 3), dtype=torch.uint8, device=DEV) for r in rigs]
    return rigs, plans, frames, panos


def _windows(rig, n, win, rng):
    pts = [(0, 0), (rig.canvas_h - win, rig.canvas_w - win)]
    while len(pts) < n:
        pts.append((int(rng.integers(0, rig.canvas_h - win + 1)), int(rng.integers(0, rig.canvas_w - win + 1))))
    return pts


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batched_tall_tiles_equal_one_by_one_and_the_oracle(storage):
    rigs, plans, frames, panos = _setup(storage)
    ref = [p.frame(f).clone() for p, f in zip(plans, frames)]
    torch.cuda.synchronize()
    b = P.Batch(plans)
    cfg0 = b.config()
    # the planner's own choice at this size is a tall tile for the level-0 pass
    assert cfg0["tile_rows"][0] >= 64, cfg0
    s = torch.cuda.Stream()
    settings = [None, ([-1] * 6, [128] * 6), ([2] * 6, [64] * 6), ([0] * 6, [16, 32, 128, 64, 16, 32]),
                ("groups", 2), ("groups", 4), ("groups", 1)]
    for st in settings:
        if st is not None and st[0] == "groups":
            b.set_groups(st[1])
            assert b.groups == st[1]
        elif st is not None:
            b.set_config(*st)
            got = b.config()
            assert got["tile_rows"][:6] == st[1] and got["wg_per_cu"][:6] == st[0]
        for p in panos:
            p.fill_(7)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.run(frames, panos, stream=s)
            b.run(frames, panos, stream=s)       # a graph replay after the capture
        s.synchronize()
        for j, (a, c) in enumerate(zip(panos, ref)):
            assert torch.equal(a, c), f"setting {st}, job {SUBSET[j]}"
    # the last batched run left every job's bands and R_0 in its plan's workspace
    rng = np.random.default_rng(11)
    got_u8, want_u8 = [], []
    r0_tol = 1e-4 if storage == "f32" else _fp16_r0_bound(7) + 1e-6
    l_tol = 1e-4 if storage == "f32" else 16 * U16
    for rig, plan, fr, pano in zip(rigs, plans, frames, panos):
        so = o.StitchOracle([f.cpu().numpy() for f in fr], rig.H, rig.masks(), rig.canvas_w, rig.canvas_h,
                            rig.levels)
        r0 = plan.view("r", 0, 0)[0]
        pano_h = pano.cpu().numpy()
        for (y, x) in _windows(rig, 6, 32, rng):
            rows, cols = np.arange(y, y + 32), np.arange(x, x + 32)
            R = so.R(0, rows, cols)
            assert_float_parity(r0[:, y:y + 32, x:x + 32].float().cpu().numpy(), R, r0_tol, f"{rig.name} R0 {(y, x)}")
            got_u8.append(pano_h[y:y + 32, x:x + 32].reshape(-1))
            want_u8.append(o.quantise(R).reshape(-1))
            so.clear()
        # bands of every camera at every level, on a window inside each band
        for i in range(rig.n):
            for k in range(rig.levels):
                lap, (ox, oy) = plan.view("lap", i, k)
                if lap is None:
                    continue
                h, w = lap.shape[1:]
                wy, wx = min(16, h), min(16, w)
                y0 = int(rng.integers(0, h - wy + 1))
                x0 = int(rng.integers(0, w - wx + 1))
                got = lap[:, y0:y0 + wy, x0:x0 + wx].float().cpu().numpy()
                want = so.Lap(i, k, np.arange(oy + y0, oy + y0 + wy), np.arange(ox + x0, ox + x0 + wx))
                assert_float_parity(got, want, l_tol, f"{rig.name} L cam{i} k{k}")
                so.clear()
    got_u8, want_u8 = np.concatenate(got_u8), np.concatenate(want_u8)
    if storage == "f32":
        assert_u8_parity(got_u8, want_u8, max_frac=1e-4)
    else:
        d = np.abs(got_u8.astype(int) - want_u8.astype(int))
        assert d.max() <= int(np.floor(255 * _fp16_r0_bound(7) + 1))


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_plain_form_settings_and_autotune_keep_the_panorama(storage, tmp_path):
    """stitch_frame under forced tile heights and grids, and after stitch_autotune (whose
    cache is then hit by a second plan), gives the default settings' panorama bit for bit."""
    rigs, plans, frames, panos = _setup(storage)
    rig, plan, fr = rigs[0], plans[0], frames[0]
    ref = plan.frame(fr).clone()
    for wg, rows in (([-1] * 6, [128] * 6), ([1] * 6, [64, 16, 32, 16, 16, 16]), ([2] * 6, [16] * 6)):
        plan.set_config(wg, rows)
        cfg = plan.config()
        assert cfg["tile_rows"][:6] == rows and cfg["wg_per_cu"][:6] == wg and not any(cfg["tile_rows"][6:])
        assert torch.equal(plan.frame(fr), ref), (wg, rows)
    cache = tmp_path / "tune.txt"
    cfg = plan.autotune(fr, cache_path=cache)
    assert all(t in (16, 32, 64, 128) for t in cfg["tile_rows"][:6])
    assert len(cache.read_text().strip().splitlines()) == 1
    assert torch.equal(plan.frame(fr), ref)
    plan2 = P.Plan(rig.frame_sizes, rig.H, rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels, storage=storage)
    assert plan2.autotune(fr, cache_path=cache) == cfg
    assert len(cache.read_text().strip().splitlines()) == 1
    assert torch.equal(plan2.frame(fr), ref)
