"""Matching and PROSAC of several area pairs with one launch per stage (stitch_lsh_match_multi,
stitch_prosac_multi; Alg. 3 for every neighbouring pair of a rig): every pair's outputs equal
the single-pair calls' bit for bit (which the other registration tests pin to the oracle),
on synthetic pairs of unequal capacities and counts and on the C2 rig's pairs as L-ORB finds
them; a second call of the same sets with other inputs reuses nothing of the first."""
import numpy as np
import pytest
import torch

import paper_1810_03988_amd as P
import workloads as wl
from oracle import register_oracle as ro
from helpers import gpu_available, rig_areas

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

ND = 256


def _pack(tern):
    n, nd = tern.shape
    w = nd // 32
    gt = (tern > 0).reshape(n, w, 32).astype(np.uint64)
    lt = (tern < 0).reshape(n, w, 32).astype(np.uint64)
    sh = np.arange(32, dtype=np.uint64)
    return np.concatenate([(gt << sh).sum(axis=2), (lt << sh).sum(axis=2)], axis=1).astype(np.uint32)


def _dev(a, dtype=torch.int32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _H(k):
    return np.array([[1.02, 0.01 * k, 200.0 + 10 * k], [-0.02, 0.99, -6.0 + k], [2e-5, -1e-5, 1.0]])


def _synthetic_pair(rng, cap_a, cap_b, count_a, count_b, k):
    """Ternary descriptors (B holds noisy copies of half of A) and points: the copies' points
    map by a projective map, the others lie at random."""
    a = rng.integers(-1, 2, (cap_a, ND))
    b = rng.integers(-1, 2, (cap_b, ND))
    n = min(count_a, count_b) // 2
    src = rng.choice(max(count_a, 1), n, replace=False)
    dst = rng.choice(max(count_b, 1), n, replace=False)
    noisy = a[src].copy()
    flip = rng.random(noisy.shape) < 0.06
    noisy[flip] = rng.integers(-1, 2, flip.sum())
    b[dst] = noisy
    pa = rng.integers(0, 600, (cap_a, 2))
    pb = rng.integers(0, 800, (cap_b, 2))
    H = _H(k)
    for s, d in zip(src, dst):
        v = H @ np.array([pa[s, 0], pa[s, 1], 1.0])
        pb[d] = np.rint(v[:2] / v[2])
    return (_dev(_pack(a).view(np.int32)), _dev([count_a]), _dev(_pack(b).view(np.int32)), _dev([count_b]),
            _dev(pa), _dev(pb))


# (cap_a, cap_b, count_a, count_b): unequal capacities, counts below them, a pair with no
# queries, a pair too small for any hypothesis, one past a 256-row key block
CASES = [(300, 420, 300, 420), (500, 260, 377, 201), (64, 64, 0, 50), (40, 90, 3, 90), (700, 650, 690, 612),
         (120, 80, 120, 80)]


def _single(inputs, pos, uni, max_dist, nhyp, T_N=200000.0, eps=3.0):
    out = []
    for da, ca, db, cb, pa, pb in inputs:
        cap_a, cap_b = da.shape[0], db.shape[0]
        m = P.Matcher(cap_a, cap_b, ND, pos, max_dist)
        m.run(da, ca, db, cb)
        pr = P.Prosac(cap_a, cap_b, nhyp, T_N, eps)
        got = pr.run(pa, pb, m.match, m.dist, ca, uni)
        out.append((m.match.cpu(), m.dist.cpu(), got))
    return out


def _multi(inputs, pos, uni, max_dist, nhyp, T_N=200000.0, eps=3.0, sets=None):
    caps = [(da.shape[0], db.shape[0]) for da, _, db, _, _, _ in inputs]
    ms, ps = sets or (P.MatcherSet(caps, ND, pos, max_dist), P.ProsacSet(caps, nhyp, T_N, eps))
    h = torch.cuda.current_stream().cuda_stream
    ms.run_raw([(da, ca, db, cb) for da, ca, db, cb, _, _ in inputs], h)
    ps.run_raw([(pa, pb, ms.match[p], ms.dist[p], ca, uni) for p, (_, ca, _, _, pa, pb) in enumerate(inputs)], h)
    torch.cuda.synchronize()
    return ms, ps


def _assert_equal(ms, ps, want):
    for p, (m, d, got) in enumerate(want):
        assert torch.equal(ms.match[p].cpu(), m), p
        assert torch.equal(ms.dist[p].cpu(), d), p
        assert np.array_equal(ps.H[p].cpu().numpy().reshape(3, 3), got["H"]), p          # bit for bit
        assert int(ps.inliers[p]) == got["inliers"], p
        assert np.array_equal(ps.mask[p].cpu().numpy().astype(bool), got["mask"]), p
        assert np.array_equal(ps.hyp_counts[p].cpu().numpy(), got["hyp_counts"]), p


def test_multi_pair_calls_equal_the_single_pair_calls():
    rng = np.random.default_rng(2024)
    inputs = [_synthetic_pair(rng, *c, k) for k, c in enumerate(CASES)]
    pos = rng.integers(0, ND, (6, 14))
    uni = _dev(np.random.default_rng(9).random((1024, 4)), torch.float64)
    want = _single(inputs, pos, uni, 64, 1024)
    ms, ps = _multi(inputs, pos, uni, 64, 1024)
    _assert_equal(ms, ps, want)
    # the pairs with enough true copies find their maps' inliers; the empty pair has none
    assert int(ps.inliers[0]) >= 60 and int(ps.inliers[4]) >= 100 and int(ps.inliers[2]) == 0
    assert (ms.match[2].cpu() == -1).all()
    # matching of pair 1 against the oracle, as a spot check of the whole set
    da, ca, db, cb = inputs[1][:4]
    wi, wd = ro.lsh_match(da.cpu().numpy().view(np.uint32)[:377], db.cpu().numpy().view(np.uint32)[:201], pos, 64)
    assert ms.match[1][:377].cpu().tolist() == wi.tolist() and ms.dist[1][:377].cpu().tolist() == wd.tolist()
    # the same sets again, on other inputs of the same capacities, in a different pair order
    # of counts: the pair tables are uploaded afresh, nothing of the first call remains
    rng2 = np.random.default_rng(77)
    inputs2 = [_synthetic_pair(rng2, a, b, max(0, ca_ - 11), cb_, k + 3) for k, (a, b, ca_, cb_) in enumerate(CASES)]
    want2 = _single(inputs2, pos, uni, 64, 1024)
    _multi(inputs2, pos, uni, 64, 1024, sets=(ms, ps))
    _assert_equal(ms, ps, want2)


def test_multi_pair_calls_on_the_c2_rig():
    """C2: L-ORB of every camera in its overlap areas (one stitch_lorb_multi call), then every
    neighbouring pair's matching and PROSAC in one call per stage; equal to the per-pair calls
    and within 1 px of the true maps on the facing areas."""
    rig = wl.rig_c2()
    areas = rig_areas(rig)
    frames = [f.cuda() for f in wl.render_rig_frames(rig)]
    pat = torch.from_numpy(wl.brief_pattern(ND)).cuda()
    ls = P.LorbSet(rig.frame_sizes, areas, n_max=500)
    ls.run_raw(frames, pat, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    first = np.cumsum([0] + [len(a) for a in areas])
    pairs = [i for i in range(rig.n - 1) if areas[i] and areas[i + 1]]
    assert len(pairs) >= 2
    inputs = []
    for i in pairs:
        za, zb = first[i] + len(areas[i]) - 1, first[i + 1]
        inputs.append((ls.descriptors[za], ls.counts[za:za + 1], ls.descriptors[zb], ls.counts[zb:zb + 1],
                       ls.points[za], ls.points[zb]))
    pos = np.random.default_rng(42).integers(0, ND, (6, 14))
    uni = _dev(np.random.default_rng(7).random((1024, 4)), torch.float64)
    want = _single(inputs, pos, uni, 64, 1024)
    ms, ps = _multi(inputs, pos, uni, 64, 1024)
    _assert_equal(ms, ps, want)
    for p, i in enumerate(pairs):
        H = ps.H[p].cpu().numpy().reshape(3, 3)
        H_true = np.linalg.inv(np.asarray(rig.H[i + 1])) @ np.asarray(rig.H[i])
        x0, y0, w, h = areas[i][-1]
        for x, y in [(x0, y0), (x0 + w, y0), (x0, y0 + h), (x0 + w, y0 + h)]:
            a, b = H @ np.array([x, y, 1.0]), H_true @ np.array([x, y, 1.0])
            assert np.hypot(*(a[:2] / a[2] - b[:2] / b[2])) < 1.0, (i, x, y)


def test_the_largest_pair_table():
    """256 pairs (the most one call takes) of small unequal capacities, some pairs empty:
    every pair's matches, PROSAC counts, inliers and map equal the single-pair calls'."""
    rng = np.random.default_rng(256)
    inputs = []
    for k in range(256):
        cap_a, cap_b = int(rng.integers(4, 48)), int(rng.integers(4, 48))
        count_a = 0 if k % 37 == 5 else int(rng.integers(0, cap_a + 1))
        inputs.append(_synthetic_pair(rng, cap_a, cap_b, count_a, int(rng.integers(1, cap_b + 1)), k % 7))
    pos = rng.integers(0, ND, (4, 10))
    uni = _dev(np.random.default_rng(3).random((64, 4)), torch.float64)
    want = _single(inputs, pos, uni, 80, 64)
    ms, ps = _multi(inputs, pos, uni, 80, 64)
    _assert_equal(ms, ps, want)


def test_all_pair_calls_replay_from_a_hip_graph():
    """Up to 16 pairs travel as kernel arguments, so both calls allocate, copy and wait for
    nothing and can be captured: three replays, with the outputs cleared by eager work and a
    synchronisation between them, each equal to the eager calls."""
    rng = np.random.default_rng(5)
    inputs = [_synthetic_pair(rng, *c, k) for k, c in enumerate(CASES)]
    pos = rng.integers(0, ND, (6, 14))
    uni = _dev(np.random.default_rng(9).random((512, 4)), torch.float64)
    ms, ps = _multi(inputs, pos, uni, 64, 512)
    outs = ms.match + ms.dist + ps.mask + [ps.H, ps.inliers, ps.hyp_counts]
    want = [t.clone() for t in outs]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=side):
        h = torch.cuda.current_stream().cuda_stream
        ms.run_raw([(da, ca, db, cb) for da, ca, db, cb, _, _ in inputs], h)
        ps.run_raw([(pa, pb, ms.match[p], ms.dist[p], ca, uni) for p, (_, ca, _, _, pa, pb) in enumerate(inputs)], h)
    for _ in range(3):
        for t in outs:
            t.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, ref in zip(outs, want):
            assert torch.equal(got, ref)


def test_validating_forms_return_the_same_results():
    """MatcherSet.run and ProsacSet.run (argument checks, host results) on the synthetic pairs."""
    rng = np.random.default_rng(31)
    inputs = [_synthetic_pair(rng, *c, k) for k, c in enumerate(CASES[:3])]
    pos = rng.integers(0, ND, (6, 14))
    uni = _dev(np.random.default_rng(4).random((256, 4)), torch.float64)
    want = _single(inputs, pos, uni, 64, 256)
    caps = [(da.shape[0], db.shape[0]) for da, _, db, _, _, _ in inputs]
    ms, ps = P.MatcherSet(caps, ND, pos, 64), P.ProsacSet(caps, 256)
    got_m = ms.run([(da, ca, db, cb) for da, ca, db, cb, _, _ in inputs])
    got_p = ps.run([(pa, pb, ms.match[p], ms.dist[p], ca, uni) for p, (_, ca, _, _, pa, pb) in enumerate(inputs)])
    for (m, d), g, (wm, wd, wg) in zip(got_m, got_p, want):
        assert torch.equal(m, wm) and torch.equal(d, wd)
        assert np.array_equal(g["H"], wg["H"]) and g["inliers"] == wg["inliers"]
        assert np.array_equal(g["mask"], wg["mask"]) and np.array_equal(g["hyp_counts"], wg["hyp_counts"])
