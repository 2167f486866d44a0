"""Pins of the registration oracle (multi-probe LSH matching, Sec. 4.2.1; PROSAC, Sec. 4.2.2)
to facts it does not compute itself: the ternary L1 distance on unpacked vectors, LSH with
one bucket against brute-force search, the probing rule, the closed form of the growth
function, exact recovery of projective maps, least-squares optimality, and PROSAC on
synthetic correspondences with outliers."""
import math

import numpy as np
import pytest

from oracle import register_oracle as ro


def _pack(tern: np.ndarray) -> np.ndarray:
    """(n, nd) values in {-1, 0, 1} -> (n, 2 nd / 32) uint32 words (gt words, lt words)."""
    n, nd = tern.shape
    out = np.zeros((n, 2 * nd // 32), dtype=np.uint32)
    for i in range(n):
        for k in range(nd):
            if tern[i, k] > 0:
                out[i, k // 32] |= np.uint32(1 << (k % 32))
            elif tern[i, k] < 0:
                out[i, nd // 32 + k // 32] |= np.uint32(1 << (k % 32))
    return out


def _tern(rng, n, nd):
    return rng.integers(-1, 2, (n, nd))


def test_distance_is_l1_of_the_ternary_vectors():
    rng = np.random.default_rng(1)
    a, b = _tern(rng, 6, 64), _tern(rng, 6, 64)
    pa, pb = _pack(a), _pack(b)
    for i in range(6):
        assert ro.distance(pa[i], pb[i]) == int(np.abs(a[i] - b[i]).sum())


def test_one_bucket_lsh_is_brute_force_nearest_neighbour():
    """k = 0: every point hashes to the one bucket, so the candidates are all points."""
    rng = np.random.default_rng(2)
    a, b = _tern(rng, 40, 64), _tern(rng, 55, 64)
    b[7] = a[3]                                      # an exact duplicate
    idx, d = ro.lsh_match(_pack(a), _pack(b), np.zeros((3, 0), dtype=np.int64), max_dist=60)
    D = np.abs(a[:, None, :] - b[None, :, :]).sum(axis=2)
    for i in range(40):
        j = int(np.argmin(D[i]))                     # argmin takes the first of equal minima
        if D[i, j] <= 60:
            assert (idx[i], d[i]) == (j, D[i, j])
        else:
            assert (idx[i], d[i]) == (-1, -1)
    assert idx[3] == 7 and d[3] == 0


def test_probing_finds_exactly_the_one_bit_neighbours():
    """The matched reference point always has a key within one bit of the query's in some
    table, and no point closer to the query (or as close with a lower index) does."""
    rng = np.random.default_rng(3)
    a, b = _tern(rng, 30, 64), _tern(rng, 80, 64)
    pa, pb = _pack(a), _pack(b)
    pos = rng.integers(0, 64, (2, 6))
    idx, d = ro.lsh_match(pa, pb, pos, max_dist=128)
    D = np.abs(a[:, None, :] - b[None, :, :]).sum(axis=2)

    def gt_bits(t, l):
        return [1 if t[p] > 0 else 0 for p in pos[l]]

    def near(i, j):
        return any(sum(x != y for x, y in zip(gt_bits(a[i], l), gt_bits(b[j], l))) <= 1 for l in range(2))

    for i in range(30):
        cands = [j for j in range(80) if near(i, j)]
        if not cands:
            assert idx[i] == -1
            continue
        best = min(cands, key=lambda j: (D[i, j], j))
        assert (idx[i], d[i]) == (best, D[i, best])


def test_growth_function_follows_its_closed_form():
    """T_n = T_N C(n, 4) / C(N, 4); T'_n - T'_{n-1} = ceil(T_n - T_{n-1}) >= 1."""
    N, T_N = 300, 200000.0
    Tp = ro.growth_schedule(N, T_N)
    C = lambda n: math.comb(n, 4)
    for n in range(5, N + 1):
        inc = Tp[n] - Tp[n - 1]
        exact = T_N * (C(n) - C(n - 1)) / C(N)
        assert inc >= 1 and abs(inc - math.ceil(exact)) <= 1
    # the increments are ceilings, so T'_N - 1 lies within N - 4 above T_N - T_4
    assert T_N - T_N / C(N) <= Tp[N] - 1 <= T_N + N
    sizes = ro.subset_sizes(N, 2000, T_N)
    ns = [n for n, _ in sizes]
    assert ns[0] == 5 and all(x <= y for x, y in zip(ns, ns[1:])) and max(ns) <= N
    # while n grows by one per hypothesis, every sample holds the newest match
    assert all(u for n, u in sizes[:20])


def test_draws_are_distinct_and_cover_the_range_ends():
    for us in ([0.0, 0.0, 0.0, 0.0], [1 - 2 ** -53] * 4, [0.5, 0.25, 0.75, 0.1]):
        got = ro.draw(us, 10, 4)
        assert len(set(got)) == 4 and all(0 <= x < 10 for x in got)
    assert ro.draw([0.0] * 4, 10, 4) == [0, 1, 2, 3]
    assert ro.draw([1 - 2 ** -53] * 4, 10, 4) == [9, 8, 7, 6]
    assert ro.sample((9, True), [0.0, 0.0, 0.0, 0.0]) == [0, 1, 2, 8]


def _H():
    return np.array([[1.02, 0.03, 210.0], [-0.02, 0.99, -6.0], [2e-5, -1e-5, 1.0]])


def _apply(H, p):
    v = H @ np.array([p[0], p[1], 1.0])
    return v[:2] / v[2]


def test_four_point_dlt_recovers_a_projective_map():
    H = _H()
    src = [(10, 20), (400, 35), (380, 300), (25, 280)]
    dst = [tuple(_apply(H, p)) for p in src]
    assert np.allclose(ro.dlt4(src, dst), H, rtol=1e-9, atol=1e-12)
    assert ro.degenerate([(0, 0), (2, 2), (5, 5), (1, 7)])
    assert not ro.degenerate(src)


def test_least_squares_dlt_is_exact_on_exact_data_and_optimal_on_noisy_data():
    H = _H()
    rng = np.random.default_rng(4)
    src = [tuple(rng.integers(0, 500, 2)) for _ in range(40)]
    dst = [tuple(_apply(H, p)) for p in src]
    assert np.allclose(ro.dlt_lsq(src, dst), H, rtol=1e-9, atol=1e-12)
    noisy = [tuple(np.array(q) + rng.normal(0, 0.5, 2)) for q in dst]
    Hl = ro.dlt_lsq(src, noisy)
    # optimality of the normalised linear least-squares objective: no coordinate step helps
    Ta, Tb = ro.normaliser(src), ro.normaliser(noisy)
    Hn = Tb @ Hl @ np.linalg.inv(Ta)
    Hn = Hn / Hn[2, 2]

    def obj(h):
        tot = 0.0
        for (x, y), (u, v) in zip(src, noisy):
            x, y, _ = Ta @ np.array([x, y, 1.0])
            u, v, _ = Tb @ np.array([u, v, 1.0])
            tot += (h[0] * x + h[1] * y + h[2] - u * (h[6] * x + h[7] * y) - u) ** 2
            tot += (h[3] * x + h[4] * y + h[5] - v * (h[6] * x + h[7] * y) - v) ** 2
        return tot

    h0 = Hn.reshape(-1)[:8]
    f0 = obj(h0)
    for k in range(8):
        for s in (1e-4, -1e-4):
            h = h0.copy()
            h[k] += s
            assert obj(h) >= f0
    assert np.abs(np.array([_apply(Hl, p) for p in src]) - np.array(dst)).max() < 1.0


def test_prosac_recovers_the_map_and_rejects_outliers():
    """120 true correspondences (integer points, targets rounded to integers) and 80
    outliers, qualities that rank most true ones first."""
    H = _H()
    rng = np.random.default_rng(5)
    n_in, n_out = 120, 80
    pa = rng.integers(0, 600, (n_in + n_out, 2))
    pb = np.array([np.rint(_apply(H, p)) for p in pa]).astype(np.int64)
    pb[n_in:] = rng.integers(0, 800, (n_out, 2))
    match_idx = np.arange(n_in + n_out)
    dist = np.concatenate([rng.integers(0, 40, n_in), rng.integers(20, 80, n_out)])
    perm = rng.permutation(n_in + n_out)
    pa, pb, dist = pa[perm], pb[perm], dist[perm]
    true_in = perm < n_in
    us = np.random.default_rng(6).random((300, 4))
    Hf, flags, counts, best = ro.prosac(pa, pb, match_idx, dist, us, 200000.0, 2.0)
    assert best >= 0 and counts[best] == counts.max()
    assert (flags & ~true_in).sum() == 0                 # outliers, all far off, rejected
    assert flags[true_in].mean() > 0.95                  # rounding moves a target <= 0.71 px
    grid = [(x, y) for x in (0, 300, 600) for y in (0, 300, 600)]
    assert max(np.hypot(*(_apply(Hf, p) - _apply(H, p))) for p in grid) < 0.6
    # too few matches: no hypothesis
    Hz, fz, cz, bz = ro.prosac(pa[:3], pb, np.arange(3), dist[:3], us, 200000.0, 2.0)
    assert bz == -1 and not fz.any() and np.all(Hz == 0)


def test_quality_order_and_match_ties_follow_the_lower_index():
    """R30/R31 tie rules: equal distances order queries by index; a query whose two nearest
    references are at equal distance takes the lower reference index."""
    order = ro.quality_order(np.array([3, -1, 0, 2, 5]), np.array([4, -1, 2, 4, 2]))
    assert order == [2, 4, 0, 3]
    rng = np.random.default_rng(8)
    a = rng.integers(-1, 2, (1, 64))
    b = np.repeat(a, 3, axis=0)
    b[0, :5] = -b[0, :5] + (b[0, :5] == 0)      # a different reference, farther away
    b[1, 0] = 1 if a[0, 0] != 1 else 0           # two references one step away
    b[2, 0] = b[1, 0]
    idx, d = ro.lsh_match(_pack(a), _pack(b), np.zeros((1, 0), dtype=np.int64), 64)
    assert idx[0] == 1 and d[0] == ro.distance(_pack(a)[0], _pack(b)[1])


def test_draws_clamp_uniforms_outside_the_unit_interval():
    assert ro.draw([-0.5, 2.0, 0.0, 0.0], 10, 2) == [0, 9]
