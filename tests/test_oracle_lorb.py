"""Pins of the L-ORB oracle (Sec. 4.1, Alg. 1-2) to facts it does not compute itself:
the segment test on a synthetic square, closed forms of the Harris response on linear
images, the BRIEF tests on a ramp, and the invariants of suppression and selection."""
import numpy as np
import pytest

from oracle import lorb_oracle as lo
import workloads as wl


def _rgb(g):
    g = np.asarray(g, dtype=np.uint8)
    return np.repeat(g[..., None], 3, axis=2)


def test_gray_is_the_integer_luma_and_exact_on_grey_frames():
    rng = np.random.default_rng(3)
    v = rng.integers(0, 256, (7, 9)).astype(np.uint8)
    assert np.array_equal(lo.gray(_rgb(v)), v)          # equal channels give the value back
    rgb = rng.integers(0, 256, (5, 6, 3)).astype(np.uint8)
    c = rgb.astype(float)
    want = np.floor((77 * c[..., 0] + 150 * c[..., 1] + 29 * c[..., 2]) / 256 + 0.5)
    assert np.array_equal(lo.gray(rgb), want.astype(np.int64))


def test_fast_finds_the_corners_of_a_square_and_not_its_edges():
    g = np.full((64, 64), 40, dtype=np.int64)
    g[20:44, 20:44] = 200
    corners = [(20, 20), (43, 20), (20, 43), (43, 43)]
    for x, y in corners:
        assert lo.fast_corner(g, x, y, 20), (x, y)
    for x, y in [(32, 20), (20, 32), (32, 43), (43, 32), (32, 32), (8, 8), (30, 50)]:
        assert not lo.fast_corner(g, x, y, 20), (x, y)
    # a single bright pixel is a corner of its dark surroundings' test, not below the threshold
    g2 = np.full((16, 16), 100, dtype=np.int64)
    g2[8, 8] = 160
    assert lo.fast_corner(g2, 8, 8, 20) and not lo.fast_corner(g2, 8, 8, 60)


@pytest.mark.parametrize("a, b", [(0, 0), (2, 3), (-3, 1), (5, 0)])
def test_harris_response_of_a_plane_is_minus_three_trace_squared(a, b):
    """g = a x + b y + c: Ix = 2a, Iy = 2b everywhere, so A = 1024 a^2, B = 1024 b^2,
    C = 1024 a b (the binomial window sums to 256), det M = 0 and R = -3 (A + B)^2."""
    y, x = np.mgrid[0:20, 0:20]
    g = a * x + b * y + 100
    A, B, C = lo.structure(g, 10, 10)
    assert (A, B, C) == (1024 * a * a, 1024 * b * b, 1024 * a * b)
    assert lo.harris(g, 10, 10) == -3 * (1024 * (a * a + b * b)) ** 2


def test_harris_response_of_a_corner_is_positive_and_of_an_edge_negative():
    g = np.full((32, 32), 50, dtype=np.int64)
    g[16:, 16:] = 180
    assert lo.harris(g, 16, 16) > 0                      # both gradients present
    assert lo.harris(g, 16, 24) < 0                      # a straight edge
    assert lo.harris(g, 6, 6) == 0                       # flat


def test_brief_on_a_ramp_orders_by_the_horizontal_offsets():
    """g = 4 x: the symmetric window gives S = 256 g, increasing in x, so the three-valued
    test of a pair is the sign of dx1 - dx2."""
    y, x = np.mgrid[0:60, 0:60]
    g = 4 * x
    S = lo.smooth(g)
    assert S[30, 30] == 256 * 4 * 30
    pat = wl.brief_pattern(256, seed=1)
    gt, lt = lo.brief(S, 30, 30, pat)
    assert np.array_equal(gt, pat[:, 0] > pat[:, 2]) and np.array_equal(lt, pat[:, 0] < pat[:, 2])
    words = lo.pack_bits(gt)
    assert words.shape == (8,) and all(((int(words[k // 32]) >> (k % 32)) & 1) == gt[k] for k in range(256))


def test_suppression_and_selection_invariants():
    rng = np.random.default_rng(11)
    g = rng.integers(0, 256, (70, 90)).astype(np.int64)
    rect = (0, 0, 90, 70)
    cand = lo.candidates(g, rect, 20, 0)
    assert cand, "random texture has corners"
    x0, y0, rw, rh = lo.clip_area(rect, 90, 70)
    assert all(x0 <= x < x0 + rw and y0 <= y < y0 + rh for x, y in cand)
    keep = lo.suppress(cand, 90)
    kset = {(x, y) for x, y, _ in keep}
    for x, y, r in keep:
        assert cand[(x, y)] == r
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                q = (x + dx, y + dy)
                if (dx or dy) and q in cand:
                    assert cand[q] <= r and q not in kset     # a maximum, and never two adjacent
    # every candidate is kept or has a neighbouring candidate at least as strong
    for (x, y), r in cand.items():
        if (x, y) not in kset:
            assert any((x + dx, y + dy) in cand and cand[(x + dx, y + dy)] >= r
                       for dx in (-1, 0, 1) for dy in (-1, 0, 1) if dx or dy)
    sel = lo.select(keep, 10, 90)
    assert len(sel) == min(10, len(keep))
    rs = [r for _, _, r in sel]
    assert rs == sorted(rs, reverse=True) and rs[0] == max(r for _, _, r in keep)


def test_lorb_output_shapes_and_margin():
    r = wl.rig_c1()
    frame = wl.render_rig_frames(r)[0].numpy()[:120, :160]
    pat = wl.brief_pattern(256)
    out = lo.lorb(frame, [(0, 0, 160, 120), (100, 40, 50, 50)], 20, 0, 25, pat)
    assert len(out) == 2
    for pts, desc in out:
        assert desc.shape == (len(pts), 16)
        for x, y, _ in pts:
            assert 17 <= x < 160 - 17 and 17 <= y < 120 - 17
    assert len(out[0][0]) == 25
    # an area past the frame clips to nothing and yields an empty, well-shaped result
    (pts, desc), = lo.lorb(frame, [(150, 10, 40, 40)], 20, 0, 25, pat)
    assert pts == [] and desc.shape == (0, 16)


def test_equal_responses_go_to_the_first_in_raster_order():
    """R23/R24 tie rules on hand-made candidates: of two adjacent candidates with equal R the
    earlier in raster order survives (also across a row boundary), and the cut at n takes
    equal responses in raster order."""
    w = 100
    cand = {(10, 5): 7, (11, 5): 7,            # same row: (10, 5) first
            (20, 8): 9, (19, 9): 9,            # (20, 8) is earlier than (19, 9) though further right
            (40, 2): 5, (60, 2): 5, (50, 1): 5, (30, 3): 5}
    keep = {(x, y) for x, y, _ in lo.suppress(cand, w)}
    assert (10, 5) in keep and (11, 5) not in keep
    assert (20, 8) in keep and (19, 9) not in keep
    sel = lo.select(lo.suppress(cand, w), 3, w)
    assert [(x, y) for x, y, _ in sel] == [(20, 8), (10, 5), (50, 1)]   # R 9, 7, then the first R 5
    sel = lo.select(lo.suppress(cand, w), 6, w)
    assert [(x, y) for x, y, _ in sel][2:] == [(50, 1), (40, 2), (60, 2), (30, 3)]


def test_threshold_keeps_a_response_equal_to_t():
    """Alg. 1, step 5 deletes the corners whose response is less than t: a FAST corner with
    R == t stays a candidate, and raising t by one removes it."""
    g = np.full((48, 48), 60, dtype=np.int64)
    g[24:, 24:] = 190
    assert lo.fast_corner(g, 24, 24, 20)
    r = lo.harris(g, 24, 24)
    rect = (20, 20, 9, 9)
    assert lo.candidates(g, rect, 20, r).get((24, 24)) == r
    assert (24, 24) not in lo.candidates(g, rect, 20, r + 1)
    assert lo.candidates(g, rect, 20, r - 1).get((24, 24)) == r
