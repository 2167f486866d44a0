"""stitch_prosac_noalloc (the allocation-free PROSAC call, scratch in a static device array)
through the C ABI against stitch_prosac with a caller workspace: two calls in a row, the
second with fewer matches and fewer hypotheses, outputs equal element by element; sizes past
the scratch are refused on the host."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1810_03988_amd as P
from helpers import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _dev(a, dtype=torch.int32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _case(seed, n, nhyp):
    H = np.array([[1.02, 0.03, 210.0], [-0.02, 0.99, -6.0], [2e-5, -1e-5, 1.0]])
    rng = np.random.default_rng(seed)
    pa = rng.integers(0, 600, (n, 2))
    v = np.c_[pa, np.ones(n)] @ H.T
    pb = np.rint(v[:, :2] / v[:, 2:]).astype(np.int64)
    k = int(0.35 * n)
    pb[n - k:] = rng.integers(0, 800, (k, 2))
    dist = rng.integers(0, 90, n)
    match = np.arange(n)
    match[::11] = -1                      # some queries without a match
    us = rng.random((nhyp, 4))
    return pa, pb, match, dist, us


def _outputs(n, nhyp):
    return (torch.zeros(9, dtype=torch.float64, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda"),
            torch.zeros(n, dtype=torch.uint8, device="cuda"), torch.zeros(nhyp, dtype=torch.int32, device="cuda"))


def _run(noalloc, pa, pb, match, dist, us, T_N=200000.0, eps=2.0):
    n, nhyp = len(pa), len(us)
    a, b, m, d, c, u = _dev(pa), _dev(pb), _dev(match), _dev(dist), _dev([n]), _dev(us, torch.float64)
    H, inl, mask, counts = _outputs(n, nhyp)
    s = torch.cuda.current_stream().cuda_stream
    lib = P.lib()
    if noalloc:
        st = lib.stitch_prosac_noalloc(a.data_ptr(), b.data_ptr(), n, m.data_ptr(), d.data_ptr(), c.data_ptr(), n,
                                       nhyp, u.data_ptr(), T_N, eps, H.data_ptr(), inl.data_ptr(), mask.data_ptr(),
                                       counts.data_ptr(), s)
    else:
        nbytes = lib.stitch_prosac_workspace_bytes(n, nhyp)
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ws = buf.data_ptr() + (-buf.data_ptr()) % 256
        st = lib.stitch_prosac(a.data_ptr(), b.data_ptr(), n, m.data_ptr(), d.data_ptr(), c.data_ptr(), n, nhyp,
                               u.data_ptr(), T_N, eps, H.data_ptr(), inl.data_ptr(), mask.data_ptr(),
                               counts.data_ptr(), ws, nbytes, s)
    assert st == 0, P.stitch.last_error()
    torch.cuda.synchronize()
    return H.cpu().numpy(), int(inl[0]), mask.cpu().numpy(), counts.cpu().numpy()


def _same(x, y):
    Hx, ix, mx, cx = x
    Hy, iy, my, cy = y
    assert np.array_equal(cx, cy) and ix == iy and np.array_equal(mx, my)
    assert np.array_equal(Hx, Hy) or np.allclose(Hx, Hy, rtol=1e-12, atol=1e-14 * np.abs(Hy).max())


def test_noalloc_equals_workspace_call_twice_in_a_row():
    big = _case(1, 900, 4096)
    small = _case(2, 150, 512)
    first = _run(True, *big)
    _same(first, _run(False, *big))
    assert first[1] >= 400
    second = _run(True, *small)             # the scratch still holds the first call's contents
    _same(second, _run(False, *small))
    assert second[1] >= 60


def test_noalloc_refuses_sizes_past_its_scratch():
    lib = P.lib()
    fake = 0x10000
    assert lib.stitch_prosac_workspace_bytes(4096, 12281) > (1 << 20)
    st = lib.stitch_prosac_noalloc(fake, fake, 100, fake, fake, fake, 4096, 12281, fake, 2e5, 2.0, fake, fake, fake,
                                   fake, None)
    assert st == 2 and "scratch" in P.stitch.last_error()
