"""stitch_detection_areas (Alg. 2 step 1, host-only) on the CPU: equal to the oracle's
areas on every workload's rigs and on random rigs, and its argument checks."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1810_03988_amd as P
from paper_1810_03988_amd import stitch as S
import workloads as wl

E = {name: i for i, name in enumerate(S.STATUS)}


def _rigs():
    out = [wl.rig_c1(), wl.rig_c2(), wl.rig_c4()]
    out += wl.rig_c3_jobs(64)
    out += wl.rig_c5_pairs(16)
    return out


@pytest.mark.parametrize("margin", [0, 24])
def test_workload_rigs_equal_the_oracle(margin):
    """C1, C2, C4, the 64 C3 jobs and the 16 C5 pairs: every frame's areas, exactly."""
    n_areas = 0
    for r in _rigs():
        got = P.detection_areas(r.frame_sizes, r.H, r.canvas_w, r.canvas_h, margin)
        want = oracle.detection_areas(r.frame_sizes, r.H, r.canvas_w, r.canvas_h, margin)
        assert got == want, r.name
        n_areas += sum(len(a) for a in got)
    assert n_areas > 200


def test_random_projective_rigs_equal_the_oracle():
    """Rows of 2-6 cameras with random sizes, small rotations, scales and perspective."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        n = int(rng.integers(2, 7))
        sizes = [(int(rng.integers(40, 700)), int(rng.integers(30, 500))) for _ in range(n)]
        Hs, x = [], 0.0
        for w, h in sizes:
            a = np.deg2rad(rng.uniform(-8, 8))
            s = rng.uniform(0.7, 1.3)
            A = np.array([[s * np.cos(a), -s * np.sin(a), x], [s * np.sin(a), s * np.cos(a), rng.uniform(-20, 20)],
                          [rng.uniform(-3e-4, 3e-4), rng.uniform(-3e-4, 3e-4), 1.0]])
            Hs.append(A)
            x += w * rng.uniform(0.6, 0.95)
        cw, ch = int(x + 800), int(max(h for _, h in sizes) + 60)
        margin = int(rng.integers(0, 40))
        got = P.detection_areas(sizes, Hs, cw, ch, margin)
        want = oracle.detection_areas(sizes, Hs, cw, ch, margin)
        assert got == want


def test_closed_form_pair():
    T = np.array([[1.0, 0, 400], [0, 1.0, 3], [0, 0, 1.0]])
    assert P.detection_areas([(640, 480)] * 2, [np.eye(3), T], 1040, 480, 24) == [[(375, 0, 265, 480)],
                                                                                [(0, 0, 265, 478)]]


def _call(n=2, fw=(640, 640), fh=(480, 480), H=None, cw=1040, ch=480, margin=24, cap=1, counts=True, areas=True):
    lib = P.lib()
    H = H if H is not None else [np.eye(3), np.array([[1.0, 0, 400], [0, 1, 3], [0, 0, 1]])]
    fwa = (ctypes.c_int32 * max(1, len(fw)))(*fw)
    fha = (ctypes.c_int32 * max(1, len(fh)))(*fh)
    ha = (ctypes.c_double * (9 * max(1, len(H))))(*[float(v) for h in H for v in np.asarray(h).reshape(9)])
    ca = (ctypes.c_int32 * max(1, n))() if counts else None
    aa = (ctypes.c_int32 * (4 * max(1, n) * max(1, cap)))() if areas else None
    return lib.stitch_detection_areas(n, fwa, fha, ha, cw, ch, margin, cap, ca, aa)


def test_argument_checks():
    assert _call() == E["OK"]
    assert _call(counts=False) == E["E_NULL"]
    assert _call(areas=False) == E["E_NULL"]
    assert _call(n=0) == E["E_SHAPE"]
    assert _call(n=65) == E["E_SHAPE"]
    assert _call(fw=(640, 0)) == E["E_SHAPE"]
    assert _call(fh=(480, 1 << 21)) == E["E_SHAPE"]
    assert _call(cw=0) == E["E_SHAPE"]
    assert _call(margin=-1) == E["E_SHAPE"]
    assert _call(cap=0) == E["E_SHAPE"]
    bad = np.eye(3)
    bad[0, 1] = np.nan
    assert _call(H=[np.eye(3), bad]) == E["E_HOMOGRAPHY"]
    # three cameras in a row: the middle frame has two areas, more than max_areas = 1
    T = lambda tx: np.array([[1.0, 0, tx], [0, 1, 0], [0, 0, 1]])
    assert _call(n=3, fw=(400,) * 3, fh=(300,) * 3, H=[T(0), T(300), T(600)], cw=1000, ch=300, cap=1) == E["E_SHAPE"]
    assert "max_areas" in S.last_error()
    assert _call(n=3, fw=(400,) * 3, fh=(300,) * 3, H=[T(0), T(300), T(600)], cw=1000, ch=300, cap=2) == E["OK"]
