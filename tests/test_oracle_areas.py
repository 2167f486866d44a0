"""Pins of the detection-area oracle (Alg. 2 step 1 under reading R37) to closed forms,
symmetry and a dense brute-force check of its defining property."""

import numpy as np
import pytest

from oracle import areas_oracle as ao

pytestmark = pytest.mark.filterwarnings("ignore")


def T(tx, ty):
    return np.array([[1.0, 0, tx], [0, 1.0, ty], [0, 0, 1.0]])


def S(s):
    return np.diag([s, s, 1.0])


def test_translation_pair_closed_form():
    """A: identity; B: translation (+400, +3); 640x480 frames, canvas 1040x480, margin 24.
    Footprints [0,640]x[0,480] and [400,1040]x[3,483] overlap on [400,640]x[3,480]; widened
    and clipped, [376,664]x[0,480]; outward rounding with the slack adds one sample at
    integer ends.  Frame A: x in [375, 640), y in [0, 480); frame B (shifted back by
    (400, 3)): x in [0, 265), y in [0, 478)."""
    got = ao.detection_areas([(640, 480)] * 2, [np.eye(3), T(400, 3)], 1040, 480, 24)
    assert got == [[(375, 0, 265, 480)], [(0, 0, 265, 478)]]


def test_margin_zero_and_large():
    got = ao.detection_areas([(640, 480)] * 2, [np.eye(3), T(400, 0)], 1040, 480, 0)
    assert got == [[(399, 0, 241, 480)], [(0, 0, 241, 480)]]
    # a margin wider than the canvas: the overlap becomes the whole canvas, so each frame's
    # area is the whole frame
    got = ao.detection_areas([(640, 480)] * 2, [np.eye(3), T(400, 0)], 1040, 480, 5000)
    assert got == [[(0, 0, 640, 480)], [(0, 0, 640, 480)]]


def test_identical_cameras_and_disjoint_and_touching():
    got = ao.detection_areas([(320, 240)] * 2, [np.eye(3), np.eye(3)], 320, 240, 8)
    assert got == [[(0, 0, 320, 240)], [(0, 0, 320, 240)]]
    # far apart: no overlap, no areas, whatever the margin
    assert ao.detection_areas([(100, 100)] * 2, [np.eye(3), T(500, 0)], 600, 100, 50) == [[], []]
    # touching along x = 100 (zero-area overlap): no areas
    assert ao.detection_areas([(100, 100)] * 2, [np.eye(3), T(100, 0)], 200, 100, 50) == [[], []]


def test_scaled_camera_closed_form():
    """B maps its 200x100 frame at scale 2 to [100, 500] x [0, 200]; A is 300x200 at the
    origin.  Overlap [100, 300] x [0, 200], margin 10 -> [90, 310] x [0, 200] (clipped to
    the 500x200 canvas).  In B (inverse: halve, then shift): x in [-5, 105], y in [0, 100]
    -> [0, 106) x [0, 100) after outward rounding and clipping; in A: [89, 300) x [0, 200)."""
    HB = T(100, 0) @ S(2.0)
    got = ao.detection_areas([(300, 200), (200, 100)], [np.eye(3), HB], 500, 200, 10)
    assert got == [[(89, 0, 211, 200)], [(0, 0, 106, 100)]]


def test_rotated_camera_closed_form():
    """B is rotated by 90 degrees (x' = -y + 300, y' = x): its 100x300 frame covers
    [0, 300] x [0, 100]; A's 300x100 frame covers the same box.  The overlap, widened by 4
    and clipped to the 300x100 canvas, is the whole canvas; mapped back into B it is the
    whole frame."""
    HB = np.array([[0, -1.0, 300], [1.0, 0, 0], [0, 0, 1.0]])
    got = ao.detection_areas([(300, 100), (100, 300)], [np.eye(3), HB], 300, 100, 4)
    assert got == [[(0, 0, 300, 100)], [(0, 0, 100, 300)]]


def test_order_and_permutation_symmetry():
    """Three cameras in a row: the middle one has two areas, ordered by partner; permuting
    the cameras permutes the result."""
    sizes = [(400, 300)] * 3
    Hs = [np.eye(3), T(300, 0), T(600, 0)]
    got = ao.detection_areas(sizes, Hs, 1000, 300, 10)
    assert len(got[0]) == 1 and len(got[1]) == 2 and len(got[2]) == 1
    assert got[1][0][0] == 0 and got[1][1][0] > 0        # partner 0 on the left, partner 2 on the right
    perm = [2, 0, 1]
    got_p = ao.detection_areas([sizes[p] for p in perm], [Hs[p] for p in perm], 1000, 300, 10)
    assert got_p[1] == got[0] and got_p[0] == got[2]
    assert sorted(got_p[2]) == sorted(got[1])


def test_unbounded_footprint_gets_no_area():
    """A homography whose depth changes sign over the frame (a camera seeing the horizon)
    has no bounded footprint: neither it nor its partner gets an area from that pair."""
    H = np.array([[1.0, 0, 0], [0, 1.0, 0], [0.01, 0, -1.0]])   # depth 0.01 x - 1 changes sign at x = 100
    assert ao.footprint(H, 200, 100) is None
    assert ao.detection_areas([(200, 100)] * 2, [np.eye(3), H], 300, 300, 5) == [[], []]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_projective_pair_brute_force(seed):
    """Random mild projective pair: every point of the widened overlap that maps into the
    frame maps into the area (dense sampling, including the overlap's corners), and every
    side of the area that the frame does not clip is within two samples of such an image."""
    rng = np.random.default_rng(seed)
    w, h = 320, 240
    HB = T(220 + rng.uniform(-10, 10), rng.uniform(-5, 5)) @ np.array(
        [[1.0 + rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), 0],
         [rng.uniform(-0.05, 0.05), 1.0 + rng.uniform(-0.05, 0.05), 0],
         [rng.uniform(-2e-4, 2e-4), rng.uniform(-2e-4, 2e-4), 1.0]])
    Hs = [np.eye(3), HB]
    m = 12
    got = ao.detection_areas([(w, h)] * 2, Hs, 560, 260, m)
    FA, FB = ao.footprint(Hs[0], w, h), ao.footprint(HB, w, h)
    ox0, oy0 = max(FA[0], FB[0]) - m, max(FA[1], FB[1]) - m
    ox1, oy1 = min(FA[2], FB[2]) + m, min(FA[3], FB[3]) + m
    ox0, oy0, ox1, oy1 = max(ox0, 0), max(oy0, 0), min(ox1, 560), min(oy1, 260)
    gx, gy = np.meshgrid(np.linspace(ox0, ox1, 61), np.linspace(oy0, oy1, 61))
    q = np.stack([gx.ravel(), gy.ravel(), np.ones(gx.size)])
    for k in (0, 1):
        (x, y, aw, ah), = got[k]
        p = np.linalg.inv(Hs[k]) @ q
        px, py = p[0] / p[2], p[1] / p[2]
        inside = (px >= 0) & (px < w) & (py >= 0) & (py < h)
        # the map is projective with positive depth: the images of the rectangle lie in the
        # bounding box of its corner images, so every sample that falls in the frame falls
        # in the area
        assert np.all((px[inside] >= x - 1e-9) & (px[inside] <= x + aw + 1e-9))
        assert np.all((py[inside] >= y - 1e-9) & (py[inside] <= y + ah + 1e-9))
        # tightness: every side the frame does not clip lies within two samples of some
        # sampled image (the grid includes the overlap's corners, whose images attain the
        # extremes of a projective image of a rectangle)
        if x > 0:
            assert px[inside].min() < x + 2
        if x + aw < w:
            assert px[inside].max() > x + aw - 2
        if y > 0:
            assert py[inside].min() < y + 2
        if y + ah < h:
            assert py[inside].max() > y + ah - 2
