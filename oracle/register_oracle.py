"""Plain CPU oracle of pairwise registration after L-ORB: multi-probe LSH matching of the
descriptors (Sec. 4.2.1; Alg. 3, step 1) and PROSAC screening with the transformation it
yields (Sec. 4.2.2; Alg. 3, step 2; Alg. 4, step 5).

TEST INFRASTRUCTURE ONLY: tests/ and bench.py may import it; the HIP product path never
does, and the two share no code, header, table or helper.

The paper names the methods (Lv et al.'s multi-probe LSH; Chum and Matas' PROSAC) but fixes
none of their parameters, the distance, the match rule or the stopping rule.  Readings
(numbered after the L-ORB oracle's R17-R26):

  R27 distance of two ternary BRIEF descriptors (R25: values 1, -1, 0 kept as a "greater"
      and a "less" bit string): the L1 distance of the {-1, 0, 1} vectors, which equals
      popcount(gt ^ gt') + popcount(lt ^ lt').
  R28 LSH family: bit sampling of the "greater" string (the locality-sensitive family of
      Hamming space).  Table l hashes a descriptor to the key whose bit b is gt bit
      P[l][b], b < k; the positions P (L x k) are an input (seeded), not part of the method.
  R29 multi-probe: in every table a query probes its own bucket and the k buckets whose key
      differs from its own in one bit (the first step of the probing sequence; for bit
      sampling all one-bit perturbations score alike).  The candidates are the union over
      tables and probes.
  R30 a query's match is its nearest candidate by (distance, reference index); it is kept
      when the distance is at most D.
  R31 PROSAC's quality order: matches by (distance, query index), ascending.
  R32 PROSAC with samples of m = 4: the growth function of Chum and Matas with T_N (an
      input): T_m = T_N prod_{i<m} (m - i) / (N - i), T_{n+1} = T_n (n + 1) / (n + 1 - m),
      T'_m = 1, T'_{n+1} = T'_n + ceil(T_{n+1} - T_n), all in FP64 in exactly this order.
      Hypothesis t = 1, 2, ...: if t = T'_n and n < N, n grows by one; then, if T'_n < t
      the sample is m draws from the top n, else the n-th match and m - 1 draws from the top
      n - 1.
  R33 the draws of hypothesis t come from four input uniforms u in [0, 1): draw k takes
      r = min(floor(u_k (R - k)), R - k - 1) in FP64 (R the size of the range; clamped at 0
      too, for inputs outside [0, 1)) and picks the r-th index of the range not drawn before,
      in increasing order.
  R34 model: the direct linear transform with h33 = 1 through the four correspondences (an
      8 x 8 linear solve in FP64).  A sample in which three points of either image are
      collinear (integer cross product 0; the points are integer pixel positions) is
      degenerate: no model, no inliers.
  R35 inlier of a model H: w = (H p)_3 > 0 and ((H p)_1 / w - q_x)^2 + ((H p)_2 / w - q_y)^2
      <= eps^2, in FP64.
  R36 stopping: the paper repeats "until a satisfactory result"; here a fixed budget of I
      hypotheses is evaluated (all at once on the GPU).  The best has the most inliers, ties
      to the earlier hypothesis.  The returned transformation is the least-squares DLT
      (h33 = 1) over the best's inliers on Hartley-normalised coordinates (centroid to the
      origin, mean distance sqrt 2), or the best's own model when it has fewer than 5
      inliers.  No valid hypothesis (fewer than 4 matches, or every sample degenerate):
      zero inliers and H = 0.
"""
from __future__ import annotations

import math

import numpy as np

M_SAMPLE = 4


# ----------------------------------------------------------------------------- matching
def distance(da: np.ndarray, db: np.ndarray) -> int:
    """R27: packed descriptors (gt words then lt words, uint32) -> L1 distance."""
    x = np.bitwise_xor(da.astype(np.uint32), db.astype(np.uint32))
    return int(sum(bin(int(v)).count("1") for v in x))


def lsh_key(desc: np.ndarray, positions: np.ndarray) -> int:
    """R28: the key of one descriptor in one table (positions: k gt-bit indices)."""
    key = 0
    for b, pos in enumerate(positions):
        bit = (int(desc[pos // 32]) >> (pos % 32)) & 1
        key |= bit << b
    return key


def lsh_match(desc_a: np.ndarray, desc_b: np.ndarray, positions: np.ndarray, max_dist: int):
    """R28-R30: for each row of desc_a, (index into desc_b or -1, distance or -1).
    positions: (L, k) int array of gt-bit indices."""
    L, k = positions.shape
    tables = []
    for l in range(L):
        buckets = {}
        for j in range(len(desc_b)):
            buckets.setdefault(lsh_key(desc_b[j], positions[l]), []).append(j)
        tables.append(buckets)
    out_idx, out_d = [], []
    for i in range(len(desc_a)):
        cand = set()
        for l in range(L):
            key = lsh_key(desc_a[i], positions[l])
            for probe in [key] + [key ^ (1 << b) for b in range(k)]:
                cand.update(tables[l].get(probe, []))
        best = None
        for j in sorted(cand):
            d = distance(desc_a[i], desc_b[j])
            if best is None or d < best[0]:
                best = (d, j)
        if best is not None and best[0] <= max_dist:
            out_idx.append(best[1])
            out_d.append(best[0])
        else:
            out_idx.append(-1)
            out_d.append(-1)
    return np.array(out_idx, dtype=np.int64), np.array(out_d, dtype=np.int64)


# ----------------------------------------------------------------------------- PROSAC
def quality_order(match_idx, match_dist):
    """R31: indices of the valid matches (queries) sorted by (distance, query index)."""
    valid = [i for i in range(len(match_idx)) if match_idx[i] >= 0]
    return sorted(valid, key=lambda i: (int(match_dist[i]), i))


def growth_schedule(N: int, T_N: float, m: int = M_SAMPLE) -> dict:
    """R32: T'_n for n = m .. N (dict n -> int)."""
    T = float(T_N)
    for i in range(m):
        T = T * float(m - i) / float(N - i)
    Tp = {m: 1}
    for n in range(m, N):
        T_next = T * float(n + 1) / float(n + 1 - m)
        Tp[n + 1] = Tp[n] + int(math.ceil(T_next - T))
        T = T_next
    return Tp


def subset_sizes(N: int, I: int, T_N: float, m: int = M_SAMPLE):
    """R32: for t = 1 .. I, (n_t, uses_nth): the subset size and whether the sample is the
    n-th match plus m - 1 draws from the top n - 1."""
    Tp = growth_schedule(N, T_N, m)
    n = m
    out = []
    for t in range(1, I + 1):
        if t == Tp[n] and n < N:
            n += 1
        out.append((n, not (Tp[n] < t)))
    return out


def draw(us, R: int, count: int):
    """R33: `count` distinct indices of range(R) from the uniforms us."""
    chosen = []
    for k in range(count):
        r = max(0, min(int(math.floor(float(us[k]) * float(R - k))), R - k - 1))
        # the r-th index of range(R) not chosen before, in increasing order
        free = [x for x in range(R) if x not in chosen]
        chosen.append(free[r])
    return chosen


def sample(t_entry, us):
    """R32-R33: indices (into the quality order) of one hypothesis' four matches."""
    n, uses_nth = t_entry
    if uses_nth:
        return draw(us, n - 1, M_SAMPLE - 1) + [n - 1]
    return draw(us, n, M_SAMPLE)


def collinear(p, q, r) -> bool:
    return (q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0]) == 0


def degenerate(pts) -> bool:
    """R34: three of the four integer points on one line."""
    for a in range(4):
        for b in range(a + 1, 4):
            for c in range(b + 1, 4):
                if collinear(pts[a], pts[b], pts[c]):
                    return True
    return False


def dlt4(src, dst) -> np.ndarray:
    """R34: H (h33 = 1) with H src_i ~ dst_i for four correspondences (8 x 8 solve)."""
    A, b = [], []
    for (x, y), (u, v) in zip(src, dst):
        A.append([x, y, 1, 0, 0, 0, -u * x, -u * y])
        b.append(u)
        A.append([0, 0, 0, x, y, 1, -v * x, -v * y])
        b.append(v)
    h = np.linalg.solve(np.array(A, dtype=np.float64), np.array(b, dtype=np.float64))
    return np.append(h, 1.0).reshape(3, 3)


def inliers(H, pa, pb, eps: float) -> np.ndarray:
    """R35: boolean inlier flags of correspondences pa[i] -> pb[i] under H."""
    out = np.zeros(len(pa), dtype=bool)
    for i, ((x, y), (u, v)) in enumerate(zip(pa, pb)):
        X = H[0, 0] * x + H[0, 1] * y + H[0, 2]
        Y = H[1, 0] * x + H[1, 1] * y + H[1, 2]
        W = H[2, 0] * x + H[2, 1] * y + H[2, 2]
        if W > 0:
            ex, ey = X / W - u, Y / W - v
            out[i] = ex * ex + ey * ey <= eps * eps
    return out


def normaliser(pts) -> np.ndarray:
    """Hartley normalisation: centroid to the origin, mean distance sqrt(2)."""
    p = np.asarray(pts, dtype=np.float64)
    c = p.mean(axis=0)
    s = math.sqrt(2.0) / np.mean(np.sqrt(((p - c) ** 2).sum(axis=1)))
    return np.array([[s, 0, -s * c[0]], [0, s, -s * c[1]], [0, 0, 1]], dtype=np.float64)


def dlt_lsq(src, dst) -> np.ndarray:
    """R36: least-squares DLT (h33 = 1) on Hartley-normalised coordinates."""
    Ta, Tb = normaliser(src), normaliser(dst)
    A, b = [], []
    for (x, y), (u, v) in zip(src, dst):
        x, y, _ = Ta @ np.array([x, y, 1.0])
        u, v, _ = Tb @ np.array([u, v, 1.0])
        A.append([x, y, 1, 0, 0, 0, -u * x, -u * y])
        b.append(u)
        A.append([0, 0, 0, x, y, 1, -v * x, -v * y])
        b.append(v)
    h = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)[0]
    Hn = np.append(h, 1.0).reshape(3, 3)
    H = np.linalg.inv(Tb) @ Hn @ Ta
    return H / H[2, 2]


def prosac(pts_a, pts_b, match_idx, match_dist, uniforms: np.ndarray, T_N: float, eps: float):
    """R31-R36 on the matches of one pair: pts_a[i] matched to pts_b[match_idx[i]].
    uniforms: (I, 4) in [0, 1).  Returns (H, inlier flags over queries, per-hypothesis
    inlier counts, best hypothesis index or -1)."""
    order = quality_order(match_idx, match_dist)
    N, I = len(order), len(uniforms)
    pa = [tuple(int(v) for v in pts_a[i]) for i in order]
    pb = [tuple(int(v) for v in pts_b[match_idx[i]]) for i in order]
    counts = np.zeros(I, dtype=np.int64)
    models = [None] * I
    if N >= M_SAMPLE:
        for t, entry in enumerate(subset_sizes(N, I, T_N)):
            idx = sample(entry, uniforms[t])
            sa, sb = [pa[i] for i in idx], [pb[i] for i in idx]
            if degenerate(sa) or degenerate(sb):
                continue
            try:
                H = dlt4(sa, sb)
            except np.linalg.LinAlgError:          # h33 = 0: not representable with h33 = 1
                continue
            models[t] = H
            counts[t] = int(inliers(H, pa, pb, eps).sum())
    flags = np.zeros(len(match_idx), dtype=bool)
    valid = [t for t in range(I) if models[t] is not None]
    if not valid:
        return np.zeros((3, 3)), flags, counts, -1
    best = max(valid, key=lambda t: (counts[t], -t))
    inl = inliers(models[best], pa, pb, eps)
    for k, i in enumerate(order):
        flags[i] = inl[k]
    if inl.sum() >= 5:
        H = dlt_lsq([pa[k] for k in range(N) if inl[k]], [pb[k] for k in range(N) if inl[k]])
    else:
        H = models[best] / models[best][2, 2]
    return H, flags, counts, best
