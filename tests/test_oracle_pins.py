"""Pins of the FP64 oracle against what the definitions and the mathematics fix.

None of these re-types the oracle's own formulas: each checks a closed form, a
hand-derived value, an invariant, a special case that reduces to a textbook
operation, or a brute-force construction built a different way.  The paper prints
no worked example for this path (its figures carry no data), so every pin is
definitional.
"""
import json
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest

import oracle as o

GOLDEN = Path(__file__).parent / "golden"


def _T(tx, ty):
    return np.array([[1.0, 0, tx], [0, 1.0, ty], [0, 0, 1.0]])


def _rand_u8(rng, h, w, c=3, hi=256):
    return rng.integers(0, hi, size=(h, w, c), dtype=np.uint8) if c else rng.integers(0, hi, (h, w), dtype=np.uint8)


def _single(frame, H, canvas_w, canvas_h, levels, coords="spec"):
    return o.StitchOracle([frame], [H], [np.full((canvas_h, canvas_w), 255, np.uint8)],
                          canvas_w, canvas_h, levels, coords)


# ----------------------------------------------------------------------------- R5 reflect-101
def test_reflect101_definition():
    n = 6
    assert o.reflect101([-2, -1, 0, 5, 6, 7], n).tolist() == [2, 1, 0, 5, 4, 3]
    with pytest.raises(ValueError):
        o.reflect101([0], 2)


# ----------------------------------------------------------------------------- R3 inverse
def test_hinv_spec_exact_cases():
    # a translation inverts to the opposite translation, a uniform scale to its reciprocal
    assert np.array_equal(o.hinv_spec(_T(400.0, 3.0)), _T(-400.0, -3.0).astype(np.float32))
    S = np.diag([2.0, 4.0, 1.0])
    assert np.array_equal(o.hinv_spec(S), np.diag([0.5, 0.25, 1.0]).astype(np.float32))
    # normalisation by adj[2,2]: scaling H does not change the result
    H = np.array([[1.1, 0.02, 5.0], [-0.03, 0.97, -2.0], [1e-4, -2e-4, 1.0]])
    assert np.array_equal(o.hinv_spec(H), o.hinv_spec(3.0 * H))
    # and it is an inverse: Hinv @ H is a multiple of I to FP32 accuracy
    P = o.hinv_spec(H).astype(np.float64) @ H
    assert np.allclose(P / P[2, 2], np.eye(3), atol=1e-6)


def test_hinv_rejects_degenerate():
    with pytest.raises(ValueError):
        o.hinv_spec(np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, np.nan]]))
    with pytest.raises(ValueError):      # adj[2,2] = h00 h11 - h01 h10 = 0
        o.hinv_spec(np.array([[1.0, 2.0, 0], [2.0, 4.0, 0], [0, 0, 1.0]]))


def test_fp32_coordinates_within_rounding_bound():
    """R3: the FP32 sequence stays within its rounding-error bound of the exact
    rational map, and is exactly right for identity and integer translations."""
    H = np.array([[0.98, 0.035, 12.25], [-0.021, 1.013, -7.5], [2.1e-4, -1.3e-4, 1.0]])
    hi32 = o.hinv_spec(H)
    rows = np.arange(0, 700, 37)
    cols = np.arange(0, 1300, 53)
    x, y, zpos = o.warp_coords(hi32, rows, cols)
    assert zpos.all()
    g = [Fraction(float(v)) for v in hi32.ravel()]   # exact values of the FP32 entries
    eps = 2.0 ** -24
    for ri, Y in enumerate(rows):
        for ci, X in enumerate(cols):
            u = g[0] * X + g[1] * Y + g[2]
            v = g[3] * X + g[4] * Y + g[5]
            z = g[6] * X + g[7] * Y + g[8]
            xe, ye = float(u / z), float(v / z)
            # 3 roundings in u (and in z), 1 in the divide: |dx| <= ~ (6 eps)(|u|+|terms|)/z
            mag_u = float((abs(g[0] * X) + abs(g[1] * Y) + abs(g[2])) / z)
            mag_v = float((abs(g[3] * X) + abs(g[4] * Y) + abs(g[5])) / z)
            zr = float((abs(g[6] * X) + abs(g[7] * Y) + abs(g[8])) / z)
            assert abs(float(x[ri, ci]) - xe) <= 8 * eps * (mag_u + abs(xe) * zr) + 1e-12
            assert abs(float(y[ri, ci]) - ye) <= 8 * eps * (mag_v + abs(ye) * zr) + 1e-12
    x, y, _ = o.warp_coords(o.hinv_spec(_T(-17.0, 9.0)), rows, cols)
    assert np.array_equal(x, (cols[None, :] + 17).astype(np.float32) + 0 * rows[:, None])
    assert np.array_equal(y, (rows[:, None] - 9).astype(np.float32) + 0 * cols[None, :])


# ----------------------------------------------------------------------------- P1, P2, P6, P7 warp
def test_p1_identity_reproduces_input():
    rng = np.random.default_rng(1)
    f = _rand_u8(rng, 37, 53)
    so = _single(f, np.eye(3), 53, 37, 3)
    assert np.array_equal(so.G(0, 0), np.moveaxis(f, -1, 0) / 255.0)
    assert np.array_equal(so.panorama(), f)


def test_p2_integer_translation_shifts_exactly():
    rng = np.random.default_rng(2)
    f = _rand_u8(rng, 30, 40)
    tx, ty = 5, -3
    so = _single(f, _T(tx, ty), 50, 34, 2)
    g0 = so.G(0, 0)
    want = np.zeros((3, 34, 50))
    for Y in range(34):
        for X in range(50):
            x, y = X - tx, Y - ty
            if 0 <= x < 40 and 0 <= y < 30:
                want[:, Y, X] = f[y, x] / 255.0
    assert np.array_equal(g0, want)


def test_p6_affine_ramp_closed_form():
    """Bilinear interpolation reproduces affine functions: on a ramp source the warp
    must equal the ramp at the exact (rational) preimage of each canvas pixel.  A wrong
    map direction or a half-pixel centre offset fails by whole pixel values."""
    h = w = 64
    ys, xs = np.mgrid[0:h, 0:w]
    f = np.stack([xs + 2 * ys, 2 * xs + ys + 3, 200 - xs - ys], axis=-1).astype(np.uint8)
    coef = [(0, 1, 2), (3, 2, 1), (200, -1, -1)]
    H = np.array([[1.05, 0.04, 9.0], [-0.03, 0.96, 6.0], [3e-4, 2e-4, 1.0]])
    so = _single(f, H, 90, 80, 1)
    g0 = so.G(0, 0)
    Hi = [Fraction(float(v)) for v in np.linalg.inv(H).ravel()]
    checked = 0
    for Y in range(80):
        for X in range(90):
            z = Hi[6] * X + Hi[7] * Y + Hi[8]
            x = float((Hi[0] * X + Hi[1] * Y + Hi[2]) / z)
            y = float((Hi[3] * X + Hi[4] * Y + Hi[5]) / z)
            if 0.001 < x < w - 1.001 and 0.001 < y < h - 1.001:
                for c, (a0, bx, cy) in enumerate(coef):
                    assert abs(g0[c, Y, X] - (a0 + bx * x + cy * y) / 255.0) < 2e-6
                checked += 1
    assert checked > 3000


def test_p7_half_pixel_shift_is_neighbour_mean():
    rng = np.random.default_rng(7)
    f = _rand_u8(rng, 12, 16)
    so = _single(f, _T(0.5, 0.0), 16, 12, 1)
    g0 = so.G(0, 0)
    src = np.moveaxis(f, -1, 0).astype(np.float64) / 255.0
    want = np.zeros_like(src)
    want[:, :, 1:] = 0.5 * (src[:, :, :-1] + src[:, :, 1:])
    want[:, :, 0] = 0.5 * src[:, :, 0]          # left tap is outside: contributes 0 (R4)
    assert np.allclose(g0, want, atol=1e-15, rtol=0)


def test_warp_constant_source_and_zero_padding():
    f = np.full((20, 30, 3), 200, np.uint8)
    H = np.array([[0.9, 0.1, 4.0], [-0.1, 0.9, 3.0], [0.0, 0.0, 1.0]])
    g0 = _single(f, H, 40, 30, 1).G(0, 0)
    x, y, _ = o.warp_coords(o.hinv_spec(H), np.arange(30), np.arange(40))
    inside = (x >= 0) & (x <= 28.999) & (y >= 0) & (y <= 18.999)
    assert np.allclose(g0[:, inside], 200 / 255.0, atol=1e-6)
    far = (x < -1) | (x >= 30) | (y < -1) | (y >= 20)
    assert np.all(g0[:, far] == 0.0)


# ----------------------------------------------------------------------------- P8 golden impulses
def test_p8_impulse_responses_match_hand_derivations():
    gold = json.loads((GOLDEN / "impulse_responses.json").read_text())
    for case in gold["reduce"]:
        n, t = case["n"], case["impulse_at"]
        img = np.zeros((1, n, n))
        img[0, t, t] = 1.0
        r = np.array(case["response_16ths"]) / 16.0
        assert np.allclose(o.reduce_full(img)[0], np.outer(r, r), atol=1e-15), case
    for case in gold["expand"]:
        n, j = case["n_fine"], case["coarse_impulse_at"]
        m = (n + 1) // 2
        g = np.zeros((1, m, m))
        g[0, j, j] = 1.0
        r = np.array(case["response_16ths"]) / 16.0
        assert np.allclose(o.expand_full(g, n, n)[0], np.outer(r, r), atol=1e-15), case


# ----------------------------------------------------------------------------- P9 dense brute force
def _fold(i, n):
    """Scalar reflect-101 written independently of the oracle."""
    while i < 0 or i > n - 1:
        if i < 0:
            i = -i
        if i > n - 1:
            i = 2 * (n - 1) - i
    return i


def _dense_reduce(n):
    w = [1, 4, 6, 4, 1]
    m = (n + 1) // 2
    R = np.zeros((m, n))
    for y in range(m):
        for a in range(5):
            R[y, _fold(2 * y + a - 2, n)] += w[a] / 16.0
    return R


def _dense_expand(n):
    w = [1, 4, 6, 4, 1]
    m = (n + 1) // 2
    E = np.zeros((n, m))
    for y in range(n):
        for a in range(5):
            t = _fold(y + a - 2, n)
            if t % 2 == 0:
                E[y, t // 2] += 2 * w[a] / 16.0
    return E


@pytest.mark.parametrize("ny,nx", [(3, 3), (4, 5), (7, 6), (9, 13), (12, 11), (13, 8)])
def test_p9_dense_operators_equal_oracle(ny, nx):
    rng = np.random.default_rng(ny * 100 + nx)
    img = rng.random((2, ny, nx))
    Ry, Rx = _dense_reduce(ny), _dense_reduce(nx)
    assert np.allclose(o.reduce_full(img), Ry @ img @ Rx.T, atol=1e-14, rtol=0)
    g = rng.random((2, (ny + 1) // 2, (nx + 1) // 2))
    Ey, Ex = _dense_expand(ny), _dense_expand(nx)
    assert np.allclose(o.expand_full(g, ny, nx), Ey @ g @ Ex.T, atol=1e-14, rtol=0)


@pytest.mark.parametrize("ny,nx,L", [(13, 11, 3), (12, 9, 2), (10, 13, 3)])
def test_p9_dense_whole_path_equals_oracle(ny, nx, L):
    """Two cameras, arbitrary partition masks, the whole blend as dense matrices."""
    rng = np.random.default_rng(ny * nx + L)
    fa, fb = _rand_u8(rng, ny, nx), _rand_u8(rng, ny, nx)
    ma = _rand_u8(rng, ny, nx, c=0)
    so = o.StitchOracle([fa, fb], [np.eye(3), np.eye(3)], [ma, 255 - ma], nx, ny, L)
    dims = o.level_dims(ny, nx, L)
    Rs = [(_dense_reduce(dims[k][0]), _dense_reduce(dims[k][1])) for k in range(L - 1)]
    Es = [(_dense_expand(dims[k][0]), _dense_expand(dims[k][1])) for k in range(L - 1)]

    def gauss(img):
        out = [img]
        for k in range(L - 1):
            out.append(Rs[k][0] @ out[-1] @ Rs[k][1].T)
        return out

    def lap(img):
        g = gauss(img)
        return [g[k] - Es[k][0] @ g[k + 1] @ Es[k][1].T for k in range(L - 1)] + [g[-1]]

    la = lap(np.moveaxis(fa, -1, 0) / 255.0)
    lb = lap(np.moveaxis(fb, -1, 0) / 255.0)
    ga = gauss(ma[None] / 255.0)
    gb = gauss((255 - ma)[None] / 255.0)
    r = ga[-1] * la[-1] + gb[-1] * lb[-1]
    for k in range(L - 2, -1, -1):
        r = ga[k] * la[k] + gb[k] * lb[k] + Es[k][0] @ r @ Es[k][1].T
    assert np.allclose(so.R(0), r, atol=1e-14, rtol=0)


# ----------------------------------------------------------------------------- P3, P5 pyramids
@pytest.mark.parametrize("ny,nx,L", [(65, 97, 5), (30, 31, 4), (48, 50, 3), (7, 9, 2)])
def test_p3_collapse_of_laplacian_is_identity(ny, nx, L):
    rng = np.random.default_rng(3)
    img = rng.random((3, ny, nx))
    assert np.max(np.abs(o.collapse(o.laplacian_pyramid(img, L)) - img)) < 1e-12


@pytest.mark.parametrize("ny,nx", [(8, 9), (30, 65), (65, 130), (34, 33)])
def test_p5_constant_image_stays_constant(ny, nx):
    c = 0.37
    img = np.full((1, ny, nx), c)
    L = 3
    for g in o.gaussian_pyramid(img, L):
        assert np.allclose(g, c, atol=1e-15, rtol=0)
    lap = o.laplacian_pyramid(img, L)
    for lk in lap[:-1]:
        assert np.max(np.abs(lk)) < 1e-15
    assert np.allclose(lap[-1], c)


def test_p5_guard_edge_replicate_border_breaks_constancy():
    """The reading matters: replacing the reflect-101 fold of EXPAND by edge replication
    (index -i -> 0, n-1+i -> n-1) makes a constant image non-constant at the border,
    while the oracle's fold keeps it exact."""
    n, c = 8, 0.37
    g = np.full((1, n // 2, n // 2), c)

    def fold_rep(i):
        return min(max(i, 0), n - 1)
    w = [1, 4, 6, 4, 1]
    E = np.zeros((n, n // 2))
    for y in range(n):
        for a in range(5):
            t = fold_rep(y + a - 2)
            if t % 2 == 0:
                E[y, t // 2] += 2 * w[a] / 16.0
    bad = E @ g[0] @ E.T
    assert np.max(np.abs(bad - c)) > 0.1
    assert np.max(np.abs(o.expand_full(g, n, n) - c)) < 1e-15


def test_p13_shift_equivariance_away_from_borders():
    rng = np.random.default_rng(13)
    L, s = 4, 8                      # a shift by 2^(L-1) keeps every level's grid phase
    big = rng.random((1, 96, 128))
    a = big[:, :, :112]
    b = big[:, :, s:112 + s]
    la, lb = o.laplacian_pyramid(a, L), o.laplacian_pyramid(b, L)
    for k in range(L):
        sk = s >> k
        m = 6 * 2 ** (L - k)         # stay clear of both borders' reflections
        assert np.allclose(la[k][:, m:-m, m + sk:-m], lb[k][:, m:-m, m:-m - sk], atol=1e-13)


# ----------------------------------------------------------------------------- P4, P10, P11, P12 blend
def test_p4_all_ones_mask_returns_frame_a():
    rng = np.random.default_rng(4)
    fa, fb = _rand_u8(rng, 24, 40), _rand_u8(rng, 24, 40)
    ones = np.full((24, 40), 255, np.uint8)
    so = o.StitchOracle([fa, fb], [np.eye(3), _T(3, 1)], [ones, 0 * ones], 40, 24, 3)
    assert np.array_equal(so.panorama(), fa)
    so = o.StitchOracle([fa, fb], [np.eye(3), _T(3, 1)], [0 * ones, ones], 40, 24, 3)
    assert np.allclose(so.R(0), so.G(1, 0), atol=1e-13, rtol=0)


def test_p10_single_level_is_alpha_blend():
    rng = np.random.default_rng(10)
    fa, fb = _rand_u8(rng, 16, 20), _rand_u8(rng, 16, 20)
    m = _rand_u8(rng, 16, 20, c=0)
    so = o.StitchOracle([fa, fb], [np.eye(3), np.eye(3)], [m, 255 - m], 20, 16, 1)
    a = np.moveaxis(fa, -1, 0) / 255.0
    b = np.moveaxis(fb, -1, 0) / 255.0
    want = (m / 255.0) * a + (1.0 - m / 255.0) * b
    assert np.allclose(so.R(0), want, atol=1e-15)


def test_p11_identical_inputs_any_partition():
    rng = np.random.default_rng(11)
    f = _rand_u8(rng, 33, 47)
    m1 = rng.integers(0, 128, (33, 47)).astype(np.uint8)
    m2 = rng.integers(0, 128, (33, 47)).astype(np.uint8)
    m3 = (255 - m1.astype(int) - m2.astype(int)).astype(np.uint8)
    so = o.StitchOracle([f, f, f], [np.eye(3)] * 3, [m1, m2, m3], 47, 33, 4)
    assert np.allclose(so.R(0), np.moveaxis(f, -1, 0) / 255.0, atol=1e-13)
    assert np.array_equal(so.panorama(), f)
    for k in range(4):
        tot = sum(so.Gm(i, k) for i in range(3))
        assert np.allclose(tot, 1.0, atol=1e-14)


def test_p12_linearity_before_quantisation():
    rng = np.random.default_rng(12)
    fa = _rand_u8(rng, 20, 30, hi=100)
    fb = _rand_u8(rng, 20, 30, hi=100)
    fa2 = _rand_u8(rng, 20, 30, hi=100)
    H = [np.eye(3), np.array([[1.0, 0.02, 4.3], [-0.01, 1.0, 0.7], [0, 0, 1.0]])]
    m = _rand_u8(rng, 20, 34, c=0)
    masks = [m, 255 - m]

    def r0(a, b):
        return o.StitchOracle([a, b], H, masks, 34, 20, 3).R(0)
    lhs = r0((fa + fa2).astype(np.uint8), (2 * fb).astype(np.uint8))
    rhs = r0(fa, fb) + r0(fa2, fb)
    assert np.allclose(lhs, rhs, atol=1e-13)


# ----------------------------------------------------------------------------- validation + windows
def test_mask_partition_and_level_checks():
    f = np.zeros((10, 10, 3), np.uint8)
    with pytest.raises(ValueError):
        o.StitchOracle([f], [np.eye(3)], [np.full((10, 10), 254, np.uint8)], 10, 10, 1)
    with pytest.raises(ValueError):      # 10 -> 5 -> 3 -> 2: the fourth level has side 2
        o.StitchOracle([f], [np.eye(3)], [np.full((10, 10), 255, np.uint8)], 10, 10, 4)


def test_window_evaluation_equals_full_canvas():
    rng = np.random.default_rng(21)
    fa, fb = _rand_u8(rng, 40, 50), _rand_u8(rng, 40, 50)
    H = [np.eye(3), np.array([[0.99, 0.03, 30.2], [-0.03, 0.99, 2.1], [1e-4, 0, 1.0]])]
    m = np.zeros((44, 80), np.uint8)
    m[:, :41] = 255
    full = o.StitchOracle([fa, fb], H, [m, 255 - m], 80, 44, 4)
    win = o.StitchOracle([fa, fb], H, [m, 255 - m], 80, 44, 4)
    rows, cols = np.arange(5, 17), np.array([0, 1, 39, 40, 41, 42, 78, 79])
    assert np.array_equal(win.R(0, rows, cols), full.R(0)[:, rows[:, None], cols[None, :]])
    for k in range(4):
        r = np.arange(min(3, full.dims[k][0]))
        assert np.array_equal(win.Lap(1, k, r, r), full.Lap(1, k)[:, r[:, None], r[None, :]])
