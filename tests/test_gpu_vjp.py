"""The plan as a differentiable function of float frames (stitch_frame_forward_f32) and its
vector-Jacobian product (stitch_frame_backward) against the FP64 VJP oracle: R_0, dl/dframes
and dl/dM of every camera, with and without direct terms on the warped frames; the
dot-product identity of the GPU's own forward and backward; determinism; the pair loss's
gradient through the VJP; and the refusal of maps beyond the gather's reach."""
import numpy as np
import pytest
import torch

import oracle as o
import paper_1810_03988_amd as P
import workloads as wl
from helpers import gpu_available, random_partition

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]
DEV = "cuda"


def _rig(seed, n=3, W=203, H=117, L=3):
    rng = np.random.default_rng(seed)
    frames, Hs, sizes = [], [], []
    for i in range(n):
        fw, fh = int(rng.integers(60, 100)), int(rng.integers(40, 80))
        sizes.append((fw, fh))
        frames.append(rng.random((3, fh, fw)).astype(np.float32))
        A = np.eye(3) + rng.normal(0, [[0.04, 0.04, 0], [0.04, 0.04, 0], [3e-4, 3e-4, 0]])
        A[0, 2] = rng.uniform(-10, W - fw + 10)
        A[1, 2] = rng.uniform(-8, H - fh + 8)
        Hs.append(A)
    masks = random_partition(rng, n, H, W, "noise" if seed % 2 else "cuts")
    return frames, Hs, masks, sizes, W, H, L


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("seed, L", [(1, 3), (2, 1), (3, 4)])
def test_forward_and_vjp_match_the_oracle(seed, L):
    frames, Hs, masks, sizes, W, H, _ = _rig(seed, L=L)
    plan = P.Plan(sizes, Hs, masks, W, H, L, bind=False)
    fo = o.FrameVjpOracle([f.astype(np.float64) for f in frames], Hs, masks, W, H, L)
    fd = [torch.from_numpy(f).to(DEV) for f in frames]
    r0 = plan.forward_f32(fd).cpu().numpy()
    want = fo.forward()
    assert np.max(np.abs(r0 - want)) <= 1e-6, np.max(np.abs(r0 - want))
    rng = np.random.default_rng(seed + 100)
    u = rng.normal(size=(3, H, W)).astype(np.float32)
    direct = [rng.normal(size=(3, H, W)).astype(np.float32), None, rng.normal(size=(3, H, W)).astype(np.float32)]
    for dg in (None, direct):
        d_frames, d_M = plan.backward(fd, torch.from_numpy(u).to(DEV),
                                      None if dg is None else [None if x is None else torch.from_numpy(x).to(DEV)
                                                               for x in dg])
        wf, wm = fo.vjp(u.astype(np.float64), None if dg is None else [None if x is None else x.astype(np.float64)
                                                                      for x in dg])
        for i in range(len(frames)):
            assert _rel(d_frames[i].cpu().numpy(), wf[i]) <= 1e-6, (i, _rel(d_frames[i].cpu().numpy(), wf[i]))
            assert _rel(d_M[i], wm[i]) <= 1e-9, (i, d_M[i], wm[i])


def test_gpu_forward_and_backward_are_transposes():
    """<F(v), u> = sum_i <v_i, J_i^T u> with the GPU's own forward and backward."""
    frames, Hs, masks, sizes, W, H, L = _rig(7, n=4)
    plan = P.Plan(sizes, Hs, masks, W, H, L, bind=False)
    rng = np.random.default_rng(8)
    v = [torch.from_numpy(rng.normal(size=f.shape).astype(np.float32)).to(DEV) for f in frames]
    u = torch.from_numpy(rng.normal(size=(3, H, W)).astype(np.float32)).to(DEV)
    lhs = float((plan.forward_f32(v).double() * u.double()).sum())
    d_frames, _ = plan.backward(v, u)
    rhs = sum(float((a.double() * b.double()).sum()) for a, b in zip(v, d_frames))
    assert abs(lhs - rhs) <= 1e-5 * max(1.0, abs(lhs)), (lhs, rhs)


def test_backward_is_deterministic():
    frames, Hs, masks, sizes, W, H, L = _rig(5)
    plan = P.Plan(sizes, Hs, masks, W, H, L, bind=False)
    fd = [torch.from_numpy(f).to(DEV) for f in frames]
    u = torch.from_numpy(np.random.default_rng(1).normal(size=(3, H, W)).astype(np.float32)).to(DEV)
    a, ma = plan.backward(fd, u)
    b, mb = plan.backward(fd, u)
    assert all(torch.equal(x, y) for x, y in zip(a, b)) and np.array_equal(ma, mb)


def test_c5_pair_loss_gradient_through_the_vjp_matches_the_oracle():
    """A full 1280x720 C5 pair: the pair loss's upstream terms fed through
    stitch_frame_backward give the pair-loss oracle's gradients (frames and the 8 corners)."""
    r = wl.rig_c5_pairs(1)[0]
    w, h = r.frame_sizes[1]
    frames = [np.moveaxis(f.numpy(), -1, 0).astype(np.float32) / np.float32(255.0) for f in wl.render_rig_frames(r)]
    H1 = np.asarray(r.H[1])
    q0 = []
    for x, y in o.corners(w, h):
        vv = H1 @ [x, y, 1.0]
        q0 += [vv[0] / vv[2], vv[1] / vv[2]]
    q0 = np.array(q0) + np.random.default_rng(4).uniform(-3, 3, 8)
    Hb = P.corners_to_h(q0, w, h)
    g = P.Grad(r.frame_sizes, r.masks(), r.canvas_w, r.canvas_h, r.levels)
    g.freeze([np.eye(3), Hb])
    fd = [torch.from_numpy(f).to(DEV) for f in frames]
    q = torch.tensor(q0, dtype=torch.float64, requires_grad=True)
    fa = fd[0].clone().requires_grad_(True)
    fb = fd[1].clone().requires_grad_(True)
    loss = P.StitchPairLoss.apply(fa, fb, q, g, np.eye(3))
    loss.backward()
    go = o.GradOracle([f.astype(np.float64) for f in frames], r.masks(), r.canvas_w, r.canvas_h, r.levels,
                      coords="spec")
    frozen = go.cells([np.eye(3), Hb])
    l_want, dq_want, df_want = go.grad_q(q0, np.eye(3), w, h, frozen)
    assert abs(float(loss) - l_want) <= 1e-9 * abs(l_want)
    assert _rel(q.grad.numpy(), dq_want) <= 1e-6, (q.grad.numpy(), dq_want)
    assert _rel(fa.grad.cpu().numpy(), df_want[0]) <= 1e-6
    assert _rel(fb.grad.cpu().numpy(), df_want[1]) <= 1e-6


def test_a_map_beyond_the_gathers_reach_is_refused():
    """A frame magnified 40 times: the transpose cannot bound its gather and the call returns
    UNSUPPORTED (the kernel only sets a flag; nothing is written out of bounds)."""
    rng = np.random.default_rng(3)
    f = rng.random((3, 12, 12)).astype(np.float32)
    Hz = np.array([[40.0, 0, 5.0], [0, 40.0, 5.0], [0, 0, 1.0]])
    W, H = 200, 150
    masks = [np.full((H, W), 255, np.uint8)]
    plan = P.Plan([(12, 12)], [Hz], masks, W, H, 2, bind=False)
    with pytest.raises(P.StitchError) as e:
        plan.backward([torch.from_numpy(f).to(DEV)], torch.ones((3, H, W), device=DEV))
    assert "E_UNSUPPORTED" in str(e.value)
