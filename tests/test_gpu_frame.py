"""GPU parity of the planned whole-frame path (stitch_frame: fused warp + pyramids +
seam-weight pyramids + blend + collapse) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as o
import paper_1810_03988_amd as P
import workloads as wl
from helpers import assert_float_parity, assert_u8_parity, gpu_available, random_partition

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]
DEV = "cuda"


def _frames_np(frames):
    return [f.cpu().numpy() if torch.is_tensor(f) else f for f in frames]


def _run(frame_sizes, Hs, masks, W, H, L, frames, storage="f32", poison=True, keep_r0=True):
    plan = P.Plan(frame_sizes, Hs, masks, W, H, L, storage=storage, keep_r0=keep_r0, bind=False)
    ws = torch.empty(plan.ws_bytes + 256, dtype=torch.uint8, device=DEV)
    if poison:
        ws.fill_(0xFF)      # NaN in every float storage: a read of unwritten memory shows
    plan.bind(ws)
    dframes = [torch.as_tensor(f).to(DEV) for f in frames]
    pano = plan.frame(dframes)
    torch.cuda.synchronize()
    return plan, pano.cpu().numpy()


def _check_intermediates(plan, so, tol=1e-4):
    """Every stored band L_k (on its window), every R_k, and the seam-weight pyramid where
    it matters, against the oracle on the same canvas indices."""
    L = plan.levels
    for i in range(plan.n):
        for k in range(L):
            lap, (ox, oy) = plan.view("lap", i, k)
            if lap is None:
                continue
            got = lap.float().cpu().numpy()
            rows, cols = np.arange(oy, oy + got.shape[1]), np.arange(ox, ox + got.shape[2])
            assert_float_parity(got, so.Lap(i, k, rows, cols), tol, f"L cam{i} k{k}")
            if k >= 1:
                gm, (mx, my) = plan.view("mask", i, k)
                g = gm.float().cpu().numpy()[0]
                roi, band = plan.regions(i, k)
                # weights are exact at least 3 samples inside an ROI edge that is not a canvas edge
                H_k, W_k = so.dims[k]
                x0 = roi[0] + (3 if roi[0] > 0 else 0)
                x1 = roi[0] + roi[2] - (3 if roi[0] + roi[2] < W_k else 0)
                y0 = roi[1] + (3 if roi[1] > 0 else 0)
                y1 = roi[1] + roi[3] - (3 if roi[1] + roi[3] < H_k else 0)
                xs = np.arange(max(x0, band[0]), min(x1, band[0] + band[2]))
                ys = np.arange(max(y0, band[1]), min(y1, band[1] + band[3]))
                if len(xs) and len(ys):
                    sub = g[ys[:, None] - my, xs[None, :] - mx]
                    assert_float_parity(sub, so.Gm(i, k, ys, xs)[0], tol, f"Gm cam{i} k{k}")
    for k in range(L):
        r, _ = plan.view("r", 0, k)
        if r is not None:
            assert_float_parity(r.float().cpu().numpy(), so.R(k), tol, f"R{k}")


def test_c1_full_frame_and_every_intermediate():
    r = wl.rig_c1()
    frames = _frames_np(wl.render_rig_frames(r))
    masks = r.masks()
    plan, pano = _run(r.frame_sizes, r.H, masks, r.canvas_w, r.canvas_h, r.levels, frames)
    so = o.StitchOracle(frames, r.H, masks, r.canvas_w, r.canvas_h, r.levels)
    assert_u8_parity(pano, so.panorama())
    _check_intermediates(plan, so)


def test_c1_is_deterministic_and_repeatable():
    r = wl.rig_c1()
    frames = [f.to(DEV) for f in wl.render_rig_frames(r)]
    plan = P.Plan(r.frame_sizes, r.H, r.masks(), r.canvas_w, r.canvas_h, r.levels)
    a = plan.frame(frames).clone()
    b = plan.frame(frames).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("offset, pad", [(3, 7), (1, 16), (8, 1)])
def test_frames_at_odd_addresses_and_pitches_give_the_same_panorama(offset, pad):
    """The source rows are read as aligned 16-byte chunks (from each row's start rounded
    down) or as unaligned 8-byte pairs: frames at odd byte addresses with odd row pitches
    must give the panorama of packed frames bit for bit."""
    r = wl.rig_c1()
    frames = [f.to(DEV) for f in wl.render_rig_frames(r)]
    plan = P.Plan(r.frame_sizes, r.H, r.masks(), r.canvas_w, r.canvas_h, r.levels)
    want = plan.frame(frames).clone()
    views = []
    for f in frames:
        h, w, _ = f.shape
        pitch = 3 * w + pad
        buf = torch.zeros(offset + h * pitch + 64, dtype=torch.uint8, device=DEV)
        v = torch.as_strided(buf, (h, w, 3), (pitch, 3, 1), offset)
        v.copy_(f)
        views.append(v)
    got = plan.frame(views)
    torch.cuda.synchronize()
    assert torch.equal(got, want)


# uint8 outputs of the small-canvas tests, held together to the 0.01 % bound at the end
RANDOM_RIG_U8 = {}


@pytest.mark.parametrize("seed", range(12))
def test_random_small_rigs(seed):
    """Odd and even canvases spanning several tiles with ragged tails, 1-3 cameras,
    projective maps, noisy or cut seam weights, 1..5 levels.  Each rig: no uint8 sample off
    by more than 1 and every float level within 1e-4; the 0.01 % bound on samples off by
    one is held over all the rigs together (a single rig holds a few thousand samples)."""
    rng = np.random.default_rng(100 + seed)
    W = int(rng.integers(40, 300))
    H = int(rng.integers(24, 200))
    n = int(rng.integers(1, 4))
    maxL = 1
    while min(-(-W // 2 ** maxL), -(-H // 2 ** maxL)) >= 3:
        maxL += 1
    L = int(rng.integers(1, maxL + 1))
    sizes, Hs, frames = [], [], []
    for i in range(n):
        fw, fh = int(rng.integers(16, W + 20)), int(rng.integers(12, H + 20))
        sizes.append((fw, fh))
        frames.append(rng.integers(0, 256, (fh, fw, 3), dtype=np.uint8))
        A = np.eye(3) + rng.normal(0, [[0.03, 0.03, 0], [0.03, 0.03, 0], [2e-4, 2e-4, 0]])
        A[0, 2] = rng.uniform(-fw / 2, W - fw / 2)
        A[1, 2] = rng.uniform(-fh / 2, H - fh / 2)
        Hs.append(A)
    masks = random_partition(rng, n, H, W, "noise" if seed % 2 else "cuts")
    plan, pano = _run(sizes, Hs, masks, W, H, L, frames)
    so = o.StitchOracle(frames, Hs, masks, W, H, L)
    want = so.panorama()
    assert_u8_parity(pano, want, max_frac=1.0)
    RANDOM_RIG_U8[seed] = (pano.reshape(-1), want.reshape(-1))
    _check_intermediates(plan, so)



def test_single_level_and_camera_outside_canvas():
    rng = np.random.default_rng(7)
    W, H = 90, 50
    frames = [rng.integers(0, 256, (50, 90, 3), dtype=np.uint8) for _ in range(3)]
    Hs = [np.eye(3), np.array([[1.0, 0.01, 3.5], [0.0, 1.0, -2.25], [0, 0, 1.0]]),
          np.array([[1.0, 0, 5000.0], [0, 1.0, 0], [0, 0, 1.0]])]          # far off the canvas
    masks = random_partition(rng, 3, H, W, "noise")
    for L in (1, 3):
        plan, pano = _run([(90, 50)] * 3, Hs, masks, W, H, L, frames)
        so = o.StitchOracle(frames, Hs, masks, W, H, L)
        want = so.panorama()
        assert_u8_parity(pano, want, max_frac=1.0)
        RANDOM_RIG_U8[("outside", L)] = (pano.reshape(-1), want.reshape(-1))
        _check_intermediates(plan, so)
        roi, band = plan.regions(2, 0)
        assert roi[2] == 0 and band[2] == 0


def test_footprint_beyond_the_horizon_is_stitched_exactly():
    rng = np.random.default_rng(8)
    W, H, L = 120, 64, 3
    frame = rng.integers(0, 256, (64, 120, 3), dtype=np.uint8)
    # w = 0.012 x - 0.5 changes sign inside the frame (x ~ 41.7): no bounded footprint
    Hp = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.012, 0.0, -0.5]])
    masks = random_partition(rng, 2, H, W, "cuts")
    plan, pano = _run([(120, 64)] * 2, [np.eye(3), Hp], masks, W, H, L, [frame, frame[::-1].copy()])
    # no bounded footprint: the roi is what the blend reads of camera 1 (its band and the
    # pyramid's reach), not limited by a footprint box
    roi, band = plan.regions(1, 0)
    assert band[2] > 0 and roi[0] <= band[0] - 8 and roi[0] + roi[2] >= min(W, band[0] + band[2] + 8)
    so = o.StitchOracle([frame, frame[::-1].copy()], [np.eye(3), Hp], masks, W, H, L)
    want = so.panorama()
    assert_u8_parity(pano, want, max_frac=1.0)
    RANDOM_RIG_U8["horizon"] = (pano.reshape(-1), want.reshape(-1))


def test_identity_rig_reproduces_the_input_exactly():
    rng = np.random.default_rng(9)
    f = rng.integers(0, 256, (77, 131, 3), dtype=np.uint8)
    masks = random_partition(rng, 2, 77, 131, "noise")
    _, pano = _run([(131, 77)] * 2, [np.eye(3), np.eye(3)], masks, 131, 77, 4, [f, f])
    assert np.array_equal(pano, f)


def test_c2_full_size_sampled_windows():
    """C2 (4 x 1920x1080 -> 6400x1080, L=6) in the benchmarked launch configuration,
    checked on windows the oracle evaluates through their dependency cones: seams,
    canvas corners and edges, frame overhangs and interior points."""
    r = wl.rig_c2()
    frames_d = wl.render_rig_frames(r, frame=0, device=DEV)
    frames = _frames_np(frames_d)
    masks = r.masks()
    plan = P.Plan(r.frame_sizes, r.H, masks, r.canvas_w, r.canvas_h, r.levels, keep_r0=True)
    pano = plan.frame(frames_d).cpu().numpy()
    r0, _ = plan.view("r", 0, 0)
    r0 = r0.cpu().numpy()
    so = o.StitchOracle(frames, r.H, masks, r.canvas_w, r.canvas_h, r.levels)
    # 64 windows of 32 x 32 (196,608 uint8 samples, so the 0.01 % bound is 19 samples):
    # canvas corners and edges, the three seams, frame overhangs, and random points
    wins = [(0, 0), (0, 6368), (1048, 0), (1048, 6368), (524, 1552), (524, 3184), (524, 4816), (7, 2500),
            (1048, 4000), (300, 100), (700, 6000), (540, 1552), (0, 1552), (1048, 3184), (0, 4816), (200, 200)]
    rng = np.random.default_rng(12)
    while len(wins) < 64:
        wins.append((int(rng.integers(0, 1080 - 32 + 1)), int(rng.integers(0, 6400 - 32 + 1))))
    got_u8, want_u8 = [], []
    for (y, x) in wins:
        rows, cols = np.arange(y, y + 32), np.arange(x, x + 32)
        R = so.R(0, rows, cols)
        assert_float_parity(r0[:, rows[:, None], cols[None, :]], R, 1e-4, f"R0 window {(y, x)}")
        got_u8.append(pano[rows[:, None], cols[None, :]])
        want_u8.append(o.quantise(R))
        so.clear()
    got_u8 = np.concatenate([g.reshape(-1) for g in got_u8])
    assert got_u8.size == 64 * 32 * 32 * 3
    assert_u8_parity(got_u8, np.concatenate([w_.reshape(-1) for w_ in want_u8]), max_frac=1e-4)


def test_small_canvases_together_hold_the_uint8_bound():
    """The random rigs, the single-level / off-canvas rig and the horizon rig: each holds a
    few thousand samples (one off-by-one is already 0.01 %), so the bound on samples off by
    one is checked over all of them together (run after them, in file order)."""
    if len([k for k in RANDOM_RIG_U8 if isinstance(k, int)]) < 12:
        pytest.skip("runs after the random rigs of this file")
    got = np.concatenate([g for g, _ in RANDOM_RIG_U8.values()])
    want = np.concatenate([w for _, w in RANDOM_RIG_U8.values()])
    assert got.size >= 100_000, got.size
    assert_u8_parity(got, want, max_frac=1e-4)
