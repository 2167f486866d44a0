"""Pins of the adjoint oracle: transposes by dot-product identities and dense matrices,
the corner parameterisation by a closed form and finite differences, and the loss
gradients by FP64 central finite differences (frozen cells and overlap)."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as wl


@pytest.mark.parametrize("ny,nx", [(3, 3), (7, 10), (12, 9), (33, 64)])
def test_transposes_satisfy_dot_product_identity(ny, nx):
    rng = np.random.default_rng(ny * 31 + nx)
    g = rng.random((2, (ny + 1) // 2, (nx + 1) // 2))
    d = rng.random((2, ny, nx))
    lhs = np.sum(o.expand_full(g, ny, nx) * d)
    assert abs(lhs - np.sum(g * o.expand_T(d))) <= 1e-12 * abs(lhs)
    f = rng.random((2, ny, nx))
    dc = rng.random((2, (ny + 1) // 2, (nx + 1) // 2))
    lhs = np.sum(o.reduce_full(f) * dc)
    assert abs(lhs - np.sum(f * o.reduce_T(dc, ny, nx))) <= 1e-12 * abs(lhs)


def test_transposes_equal_dense_transposes():
    # full 2-D check against dense Kronecker operators on a tiny grid
    ny, nx = 5, 6
    basis_c = np.eye(3 * 3).reshape(9, 1, 3, 3)
    Ed = np.stack([o.expand_full(b, ny, nx).ravel() for b in basis_c], axis=1)   # (ny*nx) x 9
    basis_f = np.eye(ny * nx).reshape(ny * nx, 1, ny, nx)
    EdT = np.stack([o.expand_T(b).ravel() for b in basis_f], axis=1)             # 9 x (ny*nx)
    assert np.allclose(EdT, Ed.T, atol=1e-15)
    Rd = np.stack([o.reduce_full(b).ravel() for b in basis_f], axis=1)           # 9 x (ny*nx)
    RdT = np.stack([o.reduce_T(b, ny, nx).ravel() for b in basis_c], axis=1)     # (ny*nx) x 9
    assert np.allclose(RdT, Rd.T, atol=1e-15)


def _pair(scale=0.125, levels=3, seed=0):
    """A C5-like pair scaled down: B = T(0.8 w, 0) K R_y(phi) K^-1 of A's frame."""
    w, h = int(1280 * scale), int(720 * scale)
    f = 733.3 * scale
    cx, cy = (w - 1) / 2, (h - 1) / 2
    K = np.array([[f, 0, cx], [0, f, cy], [0, 0, 1.0]])
    a = math.radians(1.3)
    Ry = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
    HB = np.array([[1, 0, 0.8 * w], [0, 1, 0], [0, 0, 1.0]]) @ K @ Ry @ np.linalg.inv(K)
    HB /= HB[2, 2]
    W = int(round(1.8 * w))
    rig = wl.Rig("pair", 5, seed, [(w, h), (w, h)], [np.eye(3), HB], W, h, levels, [int(round(0.9 * w))])
    frames = [np.moveaxis(fr.numpy(), -1, 0).astype(np.float64) / 255.0 for fr in wl.render_rig_frames(rig)]
    return rig, frames


def test_dlt_reproduces_a_homography_and_its_jacobian():
    rig, _ = _pair()
    w, h = rig.frame_sizes[1]
    HB = rig.H[1]
    c = o.corners(w, h)
    q = []
    for x, y in c:
        v = HB @ [x, y, 1.0]
        q += [v[0] / v[2], v[1] / v[2]]
    assert np.allclose(o.dlt_from_corners(q, w, h), HB / HB[2, 2], rtol=1e-12, atol=1e-12)
    J = o.dlt_jacobian(q, w, h)
    eps = 1e-5
    for k in range(8):
        dq = np.zeros(8)
        dq[k] = eps
        fd = (o.dlt_from_corners(np.add(q, dq), w, h) - o.dlt_from_corners(np.subtract(q, dq), w, h)).ravel() / (2 * eps)
        assert np.allclose(J[:, k], fd, rtol=1e-6, atol=1e-12)
    Jm = o.canvas_map_jacobian(HB / HB[2, 2])
    for k in range(9):
        dH = np.zeros(9)
        dH[k] = 1e-6
        Hp, Hm = (HB / HB[2, 2]).ravel() + dH, (HB / HB[2, 2]).ravel() - dH
        fd = (o.hinv_ideal(Hp.reshape(3, 3)) - o.hinv_ideal(Hm.reshape(3, 3))).ravel() / 2e-6
        assert np.allclose(Jm[:, k], fd, rtol=1e-5, atol=1e-6)   # FD noise ~ eps |M| / step


def _setup(levels=3):
    rig, frames = _pair(levels=levels)
    w, h = rig.frame_sizes[1]
    go = o.GradOracle(frames, rig.masks(), rig.canvas_w, rig.canvas_h, levels, coords="ideal")
    q_gt = []
    for x, y in o.corners(w, h):
        v = rig.H[1] @ [x, y, 1.0]
        q_gt += [v[0] / v[2], v[1] / v[2]]
    q0 = np.array(q_gt) + np.random.default_rng(3).uniform(-3, 3, 8)
    frozen = go.cells([np.eye(3), o.dlt_from_corners(q0, w, h)])
    return rig, frames, go, q0, frozen, w, h


def test_g1_corner_gradient_matches_central_differences():
    rig, frames, go, q0, frozen, w, h = _setup()
    assert frozen[1].sum() > 500          # a real overlap
    loss, dq, _ = go.grad_q(q0, np.eye(3), w, h, frozen)
    step = 1e-4
    fd = np.zeros(8)
    for k in range(8):
        e = np.zeros(8)
        e[k] = step
        lp = go.loss([np.eye(3), o.dlt_from_corners(q0 + e, w, h)], frozen)
        lm = go.loss([np.eye(3), o.dlt_from_corners(q0 - e, w, h)], frozen)
        fd[k] = (lp - lm) / (2 * step)
    assert np.linalg.norm(dq - fd) / np.linalg.norm(fd) <= 1e-6, (dq, fd)


def test_g2_source_pixel_gradient_matches_central_differences():
    rig, frames, go, q0, frozen, w, h = _setup()
    H1 = o.dlt_from_corners(q0, w, h)
    st = go.forward([np.eye(3), H1], frozen)
    d_frames, _ = go.backward(st)
    rng = np.random.default_rng(4)
    for cam in range(2):
        g = d_frames[cam]
        big = np.argwhere(np.abs(g) > 1e-3 * np.abs(g).max())
        pick = big[rng.choice(len(big), size=min(64, len(big)), replace=False)]
        for c, y, x in pick:
            saved = go.frames[cam][c, y, x]
            go.frames[cam][c, y, x] = saved + 1e-3
            lp = go.loss([np.eye(3), H1], frozen)
            go.frames[cam][c, y, x] = saved - 1e-3
            lm = go.loss([np.eye(3), H1], frozen)
            go.frames[cam][c, y, x] = saved
            fd = (lp - lm) / 2e-3
            assert abs(g[c, y, x] - fd) <= 1e-6 * abs(fd) + 1e-15, (cam, c, y, x, g[c, y, x], fd)


def test_single_level_loss_closed_form():
    """With one level the blend is the alpha blend, so the loss is
    sum over Omega of ((1-m)^2 + m^2) (A - B)^2 / (6 |Omega|)."""
    rig, frames, go, q0, frozen, w, h = _setup(levels=1)
    H1 = o.dlt_from_corners(q0, w, h)
    st = go.forward([np.eye(3), H1], frozen)
    m = rig.masks()[0] / 255.0
    A, B = st["G"]
    om = st["omega"]
    want = np.sum((((1 - m) ** 2 + m ** 2)[None] * (A - B) ** 2)[:, om]) / (6.0 * om.sum())
    assert abs(st["loss"] - want) <= 1e-12 * want


# ----------------------------------------------------------------------------- the whole path's VJP
def _rig3(seed=3, W=61, H=37, L=3):
    """Three float frames with projective maps on a small odd canvas, noisy seam weights."""
    from helpers import random_partition
    rng = np.random.default_rng(seed)
    frames_u8, Hs = [], []
    for i in range(3):
        fw, fh = int(rng.integers(24, 40)), int(rng.integers(20, 34))
        frames_u8.append(rng.integers(0, 256, (fh, fw, 3), dtype=np.uint8))
        A = np.eye(3) + rng.normal(0, [[0.03, 0.03, 0], [0.03, 0.03, 0], [4e-4, 4e-4, 0]])
        A[0, 2] = rng.uniform(-4, W - fw + 4)
        A[1, 2] = rng.uniform(-3, H - fh + 3)
        Hs.append(A)
    masks = random_partition(rng, 3, H, W, "noise")
    return frames_u8, Hs, masks, W, H, L


def test_vjp_forward_of_byte_frames_is_the_stitch_oracle():
    """F(u8/255 frames) is R_0 of the forward oracle (the same warp, pyramids and blend)."""
    fu8, Hs, masks, W, H, L = _rig3()
    fo = o.FrameVjpOracle([np.moveaxis(f, -1, 0) / 255.0 for f in fu8], Hs, masks, W, H, L)
    want = o.StitchOracle(fu8, Hs, masks, W, H, L).R(0)
    assert np.max(np.abs(fo.forward() - want)) <= 1e-12


@pytest.mark.parametrize("L", [1, 2, 4])
def test_vjp_frames_satisfy_the_dot_product_identity(L):
    """R_0 is linear in the frames (fixed maps and cells): <F(v), u> = sum_i <v_i, J_i^T u>,
    and a direct term on G_0 enters as the warp's own transpose."""
    fu8, Hs, masks, W, H, _ = _rig3(seed=4 + L)
    rng = np.random.default_rng(L)
    fo = o.FrameVjpOracle([np.moveaxis(f, -1, 0) / 255.0 for f in fu8], Hs, masks, W, H, L)
    v = [rng.normal(size=(3,) + f.shape[:2]) for f in fu8]
    u = rng.normal(size=(3, H, W))
    lhs = float(np.sum(fo.forward(frames=v) * u))
    d_frames, _ = fo.vjp(u)
    rhs = sum(float(np.sum(a * b)) for a, b in zip(v, d_frames))
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))
    g = [rng.normal(size=(3, H, W)) for _ in fu8]
    d_frames2, _ = fo.vjp(np.zeros((3, H, W)), g)
    lhs2 = sum(float(np.sum(fo._warp(vi, M, c)[0] * gi)) for vi, M, c, gi in zip(v, fo.M, fo.cells, g))
    rhs2 = sum(float(np.sum(a * b)) for a, b in zip(v, d_frames2))
    assert abs(lhs2 - rhs2) <= 1e-11 * max(1.0, abs(lhs2))


def test_vjp_maps_match_central_differences():
    """d<F, u>/dM_i against FP64 central differences of the map entries (FP64 maps, cells
    fixed, so the piece is smooth), every camera and entry."""
    fu8, Hs, masks, W, H, L = _rig3(seed=9)
    fo = o.FrameVjpOracle([np.moveaxis(f, -1, 0) / 255.0 for f in fu8], Hs, masks, W, H, L, coords="ideal")
    u = np.random.default_rng(2).normal(size=(3, H, W))
    _, d_M = fo.vjp(u)
    for i in range(3):
        M = fo.M[i]
        fd = np.zeros(9)
        for j in range(9):
            step = 1e-6 * max(abs(M.flat[j]), 1e-4)
            maps_p = [m.copy() for m in fo.M]
            maps_m = [m.copy() for m in fo.M]
            maps_p[i].flat[j] += step
            maps_m[i].flat[j] -= step
            fd[j] = (np.sum(fo.forward(maps=maps_p) * u) - np.sum(fo.forward(maps=maps_m) * u)) / (2 * step)
        an = d_M[i].ravel()
        assert np.linalg.norm(an - fd) <= 1e-6 * np.linalg.norm(fd), (i, an, fd)


def test_vjp_gives_the_pair_loss_gradient():
    """The overlap loss of a pair through the VJP (dl/dP upstream, dl/dA and dl/dB as direct
    terms on the warped frames) equals the pair-loss oracle's own adjoint."""
    rig, frames, go, q0, frozen, w, h = _setup()
    H1 = o.dlt_from_corners(q0, w, h)
    st = go.forward([np.eye(3), H1], frozen)
    d_frames, d_M = go.backward(st)
    fo = o.FrameVjpOracle(frames, [np.eye(3), H1], rig.masks(), rig.canvas_w, rig.canvas_h, rig.levels,
                          coords="ideal")
    om = st["omega"][None].astype(np.float64)
    n = st["n"]
    gP = (2.0 / (6.0 * n)) * ((st["P"] - st["G"][0]) + (st["P"] - st["G"][1])) * om
    gd = [-(2.0 / (6.0 * n)) * (st["P"] - st["G"][i]) * om for i in range(2)]
    vf, vm = fo.vjp(gP, gd)
    for a, b in zip(vf, d_frames):
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1e-30, np.max(np.abs(b))) + 1e-18
    for a, b in zip(vm, d_M):
        assert np.allclose(a, b, rtol=1e-10, atol=1e-14 * np.max(np.abs(b)))
