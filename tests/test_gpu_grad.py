"""The differentiable pair form on the GPU against the FP64 adjoint oracle (coordinates in
the forward path's FP32 sequence): loss, d loss / d frames, d loss / d M of both cameras
and d loss / d q, on a full-size registration pair and on small rigs with ragged sizes,
one to four levels and noisy seam weights; the autograd wrapper; Adam refinement."""
import numpy as np
import pytest
import torch

import oracle as o
import paper_1810_03988_amd as P
import workloads as wl
from helpers import gpu_available, random_partition

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]
DEV = "cuda"


def _float_frames(rig):
    return [f.permute(2, 0, 1).float().div(255.0).contiguous() for f in wl.render_rig_frames(rig)]


def _true_corners(rig):
    w, h = rig.frame_sizes[1]
    c = np.c_[o.corners(w, h), np.ones(4)] @ np.asarray(rig.H[1]).T
    return (c[:, :2] / c[:, 2:]).ravel()


def _rel(got, want):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


def _compare(frames_dev, Hs, masks, W, H, L, tol=1e-6):
    sizes = [(f.shape[2], f.shape[1]) for f in frames_dev]
    g = P.Grad(sizes, masks, W, H, L)
    n = g.freeze(Hs)
    loss = g.forward(frames_dev, Hs)
    d_frames, d_map = g.backward()
    torch.cuda.synchronize()
    ora = o.GradOracle([f.double().cpu().numpy() for f in frames_dev], masks, W, H, L, coords="spec")
    frozen = ora.cells(Hs)
    assert n == int(frozen[1].sum())
    st = ora.forward(Hs, frozen)
    want_frames, want_M = ora.backward(st)
    assert abs(loss - st["loss"]) <= 1e-10 * abs(st["loss"])
    for i in range(2):
        assert _rel(d_frames[i].cpu().numpy(), want_frames[i]) <= tol, f"d frame {i}"
        assert _rel(d_map[i], want_M[i]) <= tol, f"d M {i}"
    return g, loss, d_map


def test_full_registration_pair_matches_the_oracle():
    """A 1280x720 pair on the 2304x720 canvas, L = 3, at corners off by up to 3 px."""
    r = wl.rig_c5_pairs(1)[0]
    fr = _float_frames(r)
    w, h = r.frame_sizes[1]
    q0 = _true_corners(r) + r.extra["corner_noise"]
    H1 = P.corners_to_h(q0, w, h)
    g, loss, d_map = _compare([f.to(DEV) for f in fr], [np.eye(3), H1], r.masks(), r.canvas_w, r.canvas_h,
                              r.levels)
    dq = P.map_grad_to_corners(q0, w, h, d_map[1])
    ora = o.GradOracle([f.double().numpy() for f in fr], r.masks(), r.canvas_w, r.canvas_h, r.levels, coords="spec")
    _, dq_want, _ = ora.grad_q(q0, np.eye(3), w, h, ora.cells([np.eye(3), H1]))
    assert _rel(dq, dq_want) <= 1e-6


def _small_h(rng, w, h, dx):
    a = rng.uniform(-0.05, 0.05)
    H = np.array([[np.cos(a), -np.sin(a), dx], [np.sin(a), np.cos(a), rng.uniform(-3, 3)],
                  [rng.uniform(-2e-4, 2e-4), rng.uniform(-2e-4, 2e-4), 1.0]])
    return H


@pytest.mark.parametrize("L, W, H, sizes, kind", [
    (1, 61, 37, [(41, 33), (45, 35)], "noise"),
    (2, 150, 70, [(96, 64), (80, 72)], "cuts"),
    (3, 147, 83, [(97, 81), (101, 79)], "noise"),
    (4, 150, 70, [(96, 64), (80, 72)], "noise"),
])
def test_small_rigs_match_the_oracle(L, W, H, sizes, kind):
    rng = np.random.default_rng(1000 + L)
    frames = [torch.from_numpy(rng.random((3, h, w)).astype(np.float32)).to(DEV) for w, h in sizes]
    Hs = [_small_h(rng, *sizes[0], 3.0), _small_h(rng, *sizes[1], W - sizes[1][0] - 4.0)]
    masks = random_partition(rng, 2, H, W, kind)
    _compare(frames, Hs, masks, W, H, L)


def test_autograd_function_routes_the_adjoint():
    rng = np.random.default_rng(5)
    sizes = [(96, 64), (80, 72)]
    W, H, L = 150, 70, 3
    frames = [torch.from_numpy(rng.random((3, h, w)).astype(np.float32)).to(DEV).requires_grad_(True)
              for w, h in sizes]
    masks = random_partition(rng, 2, H, W, "cuts")
    Ha = _small_h(rng, *sizes[0], 3.0)
    w, h = sizes[1]
    q = torch.tensor((o.corners(w, h) + [W - w - 4.0, 1.0]).ravel(), dtype=torch.float64, requires_grad=True)
    g = P.Grad(sizes, masks, W, H, L)
    g.freeze([Ha, P.corners_to_h(q.detach().numpy(), w, h)])
    loss = P.StitchPairLoss.apply(frames[0], frames[1], q, g, Ha)
    (3.0 * loss).backward()
    # the same quantities from the pair's own adjoint (stitch_grad_backward): the autograd
    # function takes them through stitch_frame_backward from the loss's FP32 upstream terms,
    # so they agree to the FP32 rounding of those terms
    loss2 = g.forward([f.detach() for f in frames], [Ha, P.corners_to_h(q.detach().numpy(), w, h)])
    d_frames, d_map = g.backward()
    assert loss2 == float(loss)
    for f, d in zip(frames, d_frames):
        assert float((f.grad - 3.0 * d).norm() / (3.0 * d).norm()) <= 1e-6
    dq = 3.0 * P.map_grad_to_corners(q.detach().numpy(), w, h, d_map[1])
    assert np.linalg.norm(q.grad.numpy() - dq) <= 1e-6 * np.linalg.norm(dq)
    # a second forward invalidates the first loss's backward
    loss_a = P.StitchPairLoss.apply(frames[0], frames[1], q, g, Ha)
    P.StitchPairLoss.apply(frames[0], frames[1], q, g, Ha)
    with pytest.raises(RuntimeError):
        loss_a.backward()


def test_adam_refinement_moves_the_corners_towards_the_truth():
    """50 Adam steps from corners off by up to 3 px (two registration pairs)."""
    for r in wl.rig_c5_pairs(2):
        fr = [f.to(DEV) for f in _float_frames(r)]
        w, h = r.frame_sizes[1]
        qt = _true_corners(r)
        g = P.Grad(r.frame_sizes, r.masks(), r.canvas_w, r.canvas_h, r.levels)
        q, log = P.refine_pair(g, fr[0], fr[1], np.eye(3), qt + r.extra["corner_noise"], steps=50, q_true=qt)
        print(r.name, {k: (f"{v[0]:.3e}", f"{v[1]:.3f}px") for k, v in log.items()})
        assert log[50][0] < log[0][0]
        assert log[50][1] < log[0][1]


def test_backward_is_deterministic_at_moved_maps():
    """Cells frozen at one pair of maps, the loss and its adjoint taken at maps moved by a
    fraction of a pixel (as during the refinement): against the oracle with the same frozen
    cells, and two backward passes equal bit for bit (the frame adjoint is a gather)."""
    rng = np.random.default_rng(77)
    sizes, W, H, L = [(97, 81), (101, 79)], 147, 83, 3
    frames = [torch.from_numpy(rng.random((3, h, w)).astype(np.float32)).to(DEV) for w, h in sizes]
    Hs = [_small_h(rng, *sizes[0], 3.0), _small_h(rng, *sizes[1], W - sizes[1][0] - 4.0)]
    moved = [h.copy() for h in Hs]
    moved[1][0, 2] += 0.37
    moved[1][1, 2] -= 0.21
    masks = random_partition(rng, 2, H, W, "noise")
    g = P.Grad(sizes, masks, W, H, L)
    g.freeze(Hs)
    runs = []
    for _ in range(2):
        loss = g.forward(frames, moved)
        d_frames, d_map = g.backward()
        torch.cuda.synchronize()
        runs.append((loss, [d.clone().cpu() for d in d_frames], np.array(d_map, copy=True)))
    assert runs[0][0] == runs[1][0]
    for i in range(2):
        assert torch.equal(runs[0][1][i], runs[1][1][i])
    assert np.array_equal(runs[0][2], runs[1][2])
    ora = o.GradOracle([f.double().cpu().numpy() for f in frames], masks, W, H, L, coords="spec")
    st = ora.forward(moved, ora.cells(Hs))
    want_frames, want_M = ora.backward(st)
    assert abs(runs[0][0] - st["loss"]) <= 1e-10 * abs(st["loss"])
    for i in range(2):
        assert _rel(runs[0][1][i].numpy(), want_frames[i]) <= 1e-6, f"d frame {i}"
        assert _rel(runs[0][2][i], want_M[i]) <= 1e-6, f"d M {i}"
