// Pairwise registration on gfx950 after L-ORB: multi-probe LSH matching of the descriptors
// (Sec. 4.2.1; Alg. 3, step 1) and PROSAC screening with the transformation it yields
// (Sec. 4.2.2; Alg. 3, step 2; Alg. 4, step 5).
//
//   distance   L1 of the ternary descriptors = popcount(gt ^ gt') + popcount(lt ^ lt')
//   LSH        bit sampling of the "greater" string: table l's key has bit b = gt bit P[l][b]
//   probes     a query's own key and the k keys one bit away, in every table; a reference
//              point is a candidate when its key is one of them in some table
//   match      the nearest candidate by (distance, reference index), kept when <= D
//   PROSAC     m = 4, quality order (distance, query index), the growth function of Chum
//              and Matas (T_N given), draws from input uniforms, 4-point DLT (h33 = 1) in
//              FP64, degenerate samples (three collinear points) skipped, inliers by squared
//              reprojection error <= eps^2 with w > 0, a fixed budget of hypotheses, the best
//              by inlier count (ties to the earlier), then the least-squares DLT over its
//              inliers on Hartley-normalised coordinates (>= 5 inliers).
//
// Matching evaluates the probe predicate over every (query, reference) pair instead of
// building hash tables: the candidates, and hence the matches, are the same, and at the
// point counts of a detection area (hundreds to a few thousand) a wave per query scanning
// the reference keys and descriptors from L2 is faster than bucket lists.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include <algorithm>
#include <climits>
#include <cmath>

#include "stitch_internal.h"

using namespace stitch;

namespace {

constexpr int kMaxTables = 16, kMaxKeyBits = 24;
constexpr int kMaxPoints = 1 << 16;
constexpr int kMaxHyp = 1 << 16;
constexpr int kSample = 4;
constexpr int kMaxPairs = 256;

struct LshParams {
  int32_t tables, kbits, words, pad;          // words: 32-bit words per bit string (nd / 32)
  int16_t pos[kMaxTables][kMaxKeyBits];
};

__device__ __forceinline__ uint32_t key_of(const uint32_t* gt, const LshParams& P, int l) {
  uint32_t key = 0;
  for (int b = 0; b < P.kbits; ++b) {
    const int p = P.pos[l][b];
    key |= ((gt[p >> 5] >> (p & 31)) & 1u) << b;
  }
  return key;
}

// keys[l][i] of the first count rows of desc (rows of 2 * words uint32); each thread copies
// its row's "greater" words to LDS first, so the bit reads are LDS reads
__device__ __forceinline__ void lsh_keys_body(const uint32_t* __restrict__ desc, const int32_t* __restrict__ count,
                                              int cap, const LshParams& P, uint32_t* __restrict__ keys, int bx) {
  __shared__ uint32_t sRow[256][17];
  const int i = bx * 256 + threadIdx.x;
  const int n = min(*count, cap);
  if (i >= n) return;                               // no block barrier below
  const uint32_t* gt = desc + (int64_t)i * 2 * P.words;
  uint32_t* row = sRow[threadIdx.x];
  for (int w = 0; w < P.words; ++w) row[w] = gt[w];
  for (int l = 0; l < P.tables; ++l) keys[(int64_t)l * cap + i] = key_of(row, P, l);
}

__global__ void __launch_bounds__(256) k_lsh_keys(const uint32_t* __restrict__ desc, const int32_t* __restrict__ count,
                                                  int cap, const LshParams P, uint32_t* __restrict__ keys) {
  lsh_keys_body(desc, count, cap, P, keys, blockIdx.x);
}

// one wave per query: lanes stride over the reference points, then a (distance, index) min
__device__ __forceinline__ void lsh_match_body(const uint32_t* __restrict__ desc_a,
                                               const int32_t* __restrict__ count_a, int cap_a,
                                               const uint32_t* __restrict__ desc_b,
                                               const int32_t* __restrict__ count_b, int cap_b, const LshParams& P,
                                               const uint32_t* __restrict__ keys_a,
                                               const uint32_t* __restrict__ keys_b, int max_dist,
                                               int32_t* __restrict__ match, int32_t* __restrict__ dist, int bx) {
  const int lane = threadIdx.x & 63;
  const int i = bx * 4 + (threadIdx.x >> 6);
  if (i >= cap_a) return;                           // whole waves leave; no block barrier below
  const int na = min(*count_a, cap_a), nb = min(*count_b, cap_b);
  if (i >= na) {
    if (lane == 0) {
      match[i] = -1;
      dist[i] = -1;
    }
    return;
  }
  const int W2 = 2 * P.words;
  uint32_t ka[kMaxTables];
  for (int l = 0; l < P.tables; ++l) ka[l] = keys_a[(int64_t)l * cap_a + i];
  const uint32_t* da = desc_a + (int64_t)i * W2;
  unsigned long long best = ~0ull;                  // (distance << 32) | index
  for (int j = lane; j < nb; j += 64) {
    bool cand = false;
    for (int l = 0; l < P.tables && !cand; ++l) cand = __popc(ka[l] ^ keys_b[(int64_t)l * cap_b + j]) <= 1;
    if (!cand) continue;
    const uint32_t* db = desc_b + (int64_t)j * W2;
    int d = 0;
    for (int w = 0; w < W2; w += 2) {                 // rows hold an even number of words
      const uint2 x = *reinterpret_cast<const uint2*>(da + w), y = *reinterpret_cast<const uint2*>(db + w);
      d += __popc(x.x ^ y.x) + __popc(x.y ^ y.y);
    }
    const unsigned long long kd = ((unsigned long long)d << 32) | (uint32_t)j;
    best = kd < best ? kd : best;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o);
    best = other < best ? other : best;
  }
  if (lane == 0) {
    const int d = (int)(best >> 32);
    const bool ok = best != ~0ull && d <= max_dist;
    match[i] = ok ? (int)(uint32_t)best : -1;
    dist[i] = ok ? d : -1;
  }
}

__global__ void __launch_bounds__(256) k_lsh_match(const uint32_t* __restrict__ desc_a,
                                                   const int32_t* __restrict__ count_a, int cap_a,
                                                   const uint32_t* __restrict__ desc_b,
                                                   const int32_t* __restrict__ count_b, int cap_b, const LshParams P,
                                                   const uint32_t* __restrict__ keys_a,
                                                   const uint32_t* __restrict__ keys_b, int max_dist,
                                                   int32_t* __restrict__ match, int32_t* __restrict__ dist) {
  lsh_match_body(desc_a, count_a, cap_a, desc_b, count_b, cap_b, P, keys_a, keys_b, max_dist, match, dist, blockIdx.x);
}

// Several pairs per launch: blockIdx.y selects the pair (keys: pair y / 2, side y % 2), its
// descriptor read from a device table; blocks past a pair's own extent leave at once.
struct LshPairDev {
  const uint32_t* desc_a;
  const int32_t* count_a;
  const uint32_t* desc_b;
  const int32_t* count_b;
  uint32_t* keys_a;
  uint32_t* keys_b;
  int32_t* match;
  int32_t* dist;
  int32_t cap_a, cap_b;
};

// Up to kArgPairs pairs travel as a kernel argument (taken at launch: no upload and no host
// wait, and the launch can be captured into a graph); more come from a device table.
constexpr int kArgPairs = 16;
template <typename D>
struct PairArgs {
  D p[kArgPairs];
};
template <typename D>
__device__ __forceinline__ D pair_of(const D* __restrict__ table, const PairArgs<D>& args, int i) {
  D q;
  if (table) q = table[i];
  else q = args.p[i];
  return q;
}

__global__ void __launch_bounds__(256) k_lsh_keys_multi(const LshPairDev* __restrict__ pairs,
                                                        const PairArgs<LshPairDev> args, const LshParams P) {
  const LshPairDev q = pair_of(pairs, args, blockIdx.y >> 1);
  const bool b = blockIdx.y & 1;
  const int cap = b ? q.cap_b : q.cap_a;
  if ((int)blockIdx.x * 256 >= cap) return;
  lsh_keys_body(b ? q.desc_b : q.desc_a, b ? q.count_b : q.count_a, cap, P, b ? q.keys_b : q.keys_a, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_lsh_match_multi(const LshPairDev* __restrict__ pairs,
                                                         const PairArgs<LshPairDev> args, const LshParams P,
                                                         int max_dist) {
  const LshPairDev q = pair_of(pairs, args, blockIdx.y);
  if ((int)blockIdx.x * 4 >= q.cap_a) return;
  lsh_match_body(q.desc_a, q.count_a, q.cap_a, q.desc_b, q.count_b, q.cap_b, P, q.keys_a, q.keys_b, max_dist, q.match,
                 q.dist, blockIdx.x);
}

// ---------------------------------------------------------------------------- PROSAC
struct ProsacWs {            // offsets into the workspace
  size_t misc, qa, qb, qi, tp, hyp_h, hyp_ok;
};

// misc: [0] M = number of matches
// one block of 1024 threads: matches in quality order, and T'_n for n = 4 .. M
__device__ __forceinline__ void prosac_prepare_body(const int32_t* __restrict__ pts_a,
                                                    const int32_t* __restrict__ pts_b, int cap_b,
                                                    const int32_t* __restrict__ match,
                                                    const int32_t* __restrict__ dist,
                                                    const int32_t* __restrict__ count_a, int cap_a, double T_N,
                                                    int32_t* __restrict__ misc, int2* __restrict__ qa,
                                                    int2* __restrict__ qb, int32_t* __restrict__ qi,
                                                    int64_t* __restrict__ tp) {
  constexpr int kStage = 16384;                      // ranking keys staged in LDS up to here
  __shared__ int sM;
  __shared__ __attribute__((aligned(16))) int32_t sKey[kStage];
  const int tid = threadIdx.x;
  const int na = min(*count_a, cap_a);
  // ranking key of query j: its distance when it has a match (below INT32_MAX), else
  // INT32_MAX, which precedes nothing and equals no valid key
  auto key = [&](int j) -> int {
    const int mj = match[j];
    return (mj >= 0 && mj < cap_b) ? min(dist[j], INT32_MAX - 1) : INT32_MAX;
  };
  const bool staged = na <= kStage;
  const int npad = (na + 3) & ~3;
  if (tid == 0) sM = 0;
  if (staged)
    for (int j = tid; j < npad; j += 1024) sKey[j] = j < na ? key(j) : INT32_MAX;
  __syncthreads();
  // number of valid matches
  int local = 0;
  for (int i = tid; i < na; i += 1024) local += key(i) != INT32_MAX;
  atomicAdd(&sM, local);
  __syncthreads();
  const int M = sM;
  // the growth function, sequentially in FP64 in the order of its definition, on the last
  // wave's last lane while the others rank the matches
  if (tid == 1023 && M >= kSample) {
    double T = T_N;
    for (int i = 0; i < kSample; ++i) T = T * (double)(kSample - i) / (double)(M - i);
    tp[kSample] = 1;
    for (int n = kSample; n < M; ++n) {
      const double Tn = T * (double)(n + 1) / (double)(n + 1 - kSample);
      tp[n + 1] = tp[n] + (int64_t)ceil(Tn - T);
      T = Tn;
    }
  }
  if (tid == 0) misc[0] = M;
  // rank of match i: the valid matches ordered before it by (distance, query index)
  for (int i = tid; i < na; i += 1024) {
    const int ki = key(i);
    if (ki == INT32_MAX) continue;
    int r = 0;
    if (staged) {
      for (int j = 0; j < npad; j += 4) {
        const int4 v = *reinterpret_cast<const int4*>(&sKey[j]);
        r += (v.x < ki || (v.x == ki && j < i)) + (v.y < ki || (v.y == ki && j + 1 < i)) +
             (v.z < ki || (v.z == ki && j + 2 < i)) + (v.w < ki || (v.w == ki && j + 3 < i));
      }
    } else {
      for (int j = 0; j < na; ++j) {
        const int kj = key(j);
        r += kj < ki || (kj == ki && j < i);
      }
    }
    const int mi = match[i];
    qa[r] = make_int2(pts_a[2 * i], pts_a[2 * i + 1]);
    qb[r] = make_int2(pts_b[2 * mi], pts_b[2 * mi + 1]);
    qi[r] = i;
  }
}

__global__ void __launch_bounds__(1024) k_prosac_prepare(const int32_t* __restrict__ pts_a,
                                                         const int32_t* __restrict__ pts_b, int cap_b,
                                                         const int32_t* __restrict__ match,
                                                         const int32_t* __restrict__ dist,
                                                         const int32_t* __restrict__ count_a, int cap_a, double T_N,
                                                         int32_t* __restrict__ misc, int2* __restrict__ qa,
                                                         int2* __restrict__ qb, int32_t* __restrict__ qi,
                                                         int64_t* __restrict__ tp) {
  prosac_prepare_body(pts_a, pts_b, cap_b, match, dist, count_a, cap_a, T_N, misc, qa, qb, qi, tp);
}

__device__ __forceinline__ bool collinear(int2 p, int2 q, int2 r) {
  return (int64_t)(q.x - p.x) * (r.y - p.y) - (int64_t)(q.y - p.y) * (r.x - p.x) == 0;
}

__device__ bool degenerate4(const int2* p) {
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b)
      for (int c = b + 1; c < 4; ++c)
        if (collinear(p[a], p[b], p[c])) return true;
  return false;
}

// Solve the 8 x 8 system A x = b with one wave: lane l holds a = A[l / 8][l % 8] and bv =
// b[l / 8].  Gaussian elimination with partial pivoting (largest |pivot|, the first row on
// ties) by shuffles, then back substitution; returns x[l % 8] in every lane, and false (in
// every lane) when a pivot is zero.
__device__ bool wave_solve8(double a, double bv, double& x_mine) {
  const int lane = threadIdx.x & 63, r = lane >> 3, c = lane & 7;
  for (int k = 0; k < 8; ++k) {
    // pivot: max |A[row][k]| over rows >= k, the first row on ties
    double v = (c == k && r >= k) ? fabs(a) : -1.0;
    int pr = r;
    for (int o = 32; o > 0; o >>= 1) {
      const double v2 = __shfl_xor(v, o);
      const int r2 = __shfl_xor(pr, o);
      if (v2 > v || (v2 == v && r2 < pr)) {
        v = v2;
        pr = r2;
      }
    }
    if (!(v > 0.0)) return false;
    // swap rows pr and k
    const int src = r == k ? pr * 8 + c : r == pr ? k * 8 + c : lane;
    a = __shfl(a, src);
    bv = __shfl(bv, src);
    const double piv = __shfl(a, k * 8 + k), prow = __shfl(a, k * 8 + c), bk = __shfl(bv, k * 8);
    const double col = __shfl(a, r * 8 + k);
    if (r > k) {
      const double f = col / piv;
      if (c >= k) a -= f * prow;
      bv -= f * bk;
    }
  }
  x_mine = 0.0;
  for (int k = 7; k >= 0; --k) {
    double t = (r == k && c > k) ? a * x_mine : 0.0;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    const double xk = (__shfl(bv, k * 8) - t) / __shfl(a, k * 8 + k);
    if (c == k) x_mine = xk;
  }
  return true;
}

// squared reprojection test in the order of its definition (no contraction)
__device__ __forceinline__ bool is_inlier(const double* H, int2 p, int2 q, double eps2) {
#pragma clang fp contract(off)
  const double x = p.x, y = p.y;
  const double X = H[0] * x + H[1] * y + H[2];
  const double Y = H[3] * x + H[4] * y + H[5];
  const double W = H[6] * x + H[7] * y + H[8];
  if (!(W > 0.0)) return false;
  const double ex = X / W - (double)q.x, ey = Y / W - (double)q.y;
  return ex * ex + ey * ey <= eps2;
}

// r-th index of [0, R) not in chosen[0 .. nch), in increasing order
__device__ int nth_free(int r, const int* chosen, int nch) {
  int s[3];
  for (int k = 0; k < nch; ++k) s[k] = chosen[k];
  for (int a = 0; a < nch; ++a)                       // sort (at most 3)
    for (int b = a + 1; b < nch; ++b)
      if (s[b] < s[a]) {
        const int t = s[a];
        s[a] = s[b];
        s[b] = t;
      }
  for (int k = 0; k < nch; ++k)
    if (s[k] <= r) ++r;
  return r;
}

// rows of the DLT system (h33 = 1) for a correspondence (x, y) -> (u, v):
//   r0 = [x, y, 1, 0, 0, 0, -u x, -u y] (right side u), r1 = [0, 0, 0, x, y, 1, -v x, -v y] (v)
__device__ __forceinline__ double row0(int i, double x, double y, double u) {
  return i == 0 ? x : i == 1 ? y : i == 2 ? 1.0 : i == 6 ? -u * x : i == 7 ? -u * y : 0.0;
}
__device__ __forceinline__ double row1(int i, double x, double y, double v) {
  return i == 3 ? x : i == 4 ? y : i == 5 ? 1.0 : i == 6 ? -v * x : i == 7 ? -v * y : 0.0;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one wave per hypothesis t: its sample, its model and its inlier count
__device__ __forceinline__ void prosac_hyp_body(const int32_t* __restrict__ misc, const int2* __restrict__ qa,
                                                const int2* __restrict__ qb, const int64_t* __restrict__ tp,
                                                int nhyp, const double* __restrict__ uniforms, double eps2,
                                                double* __restrict__ hyp_h, int32_t* __restrict__ hyp_ok,
                                                int32_t* __restrict__ hyp_counts, int bx) {
  __shared__ double sH[4][9];
  __shared__ int sOk[4];
  __shared__ int2 sPts[4][8];                         // the sample: 4 points of A, then of B
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = bx * 4 + wv;                          // hypothesis t + 1 of the schedule
  if (t >= nhyp) return;                              // whole waves; no block barrier below
  const int M = misc[0];
  if (M < kSample) {
    if (lane == 0) {
      hyp_ok[t] = 0;
      hyp_counts[t] = 0;
    }
    return;
  }
  if (lane == 0) {
    // n_t = 4 + #{n in [4, M-1] : T'_n <= t+1}: binary search over the increasing T'
    const int64_t tt = t + 1;
    int lo = kSample, hi = M;                         // first n in [4, M) with T'_n > tt, or M
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (tp[mid] <= tt) lo = mid + 1;
      else hi = mid;
    }
    const int n = kSample + (lo - kSample);
    const bool nth = !(tp[n] < tt);
    const double* u = uniforms + (int64_t)t * 4;
    int idx[4];
    const int R = nth ? n - 1 : n, draws = nth ? 3 : 4;
    for (int k = 0; k < draws; ++k) {
      // clamped into the range (uniforms outside [0, 1), even NaN, cannot index outside it)
      const double f = floor(u[k] * (double)(R - k));
      const int r = f >= 0.0 ? (int)fmin(f, (double)(R - k - 1)) : 0;
      idx[k] = nth_free(r, idx, k);
    }
    if (nth) idx[3] = n - 1;
    int2 pa[4], pb[4];
    for (int k = 0; k < 4; ++k) {
      pa[k] = qa[idx[k]];
      pb[k] = qb[idx[k]];
      sPts[wv][k] = pa[k];
      sPts[wv][4 + k] = pb[k];
    }
    sOk[wv] = !degenerate4(pa) && !degenerate4(pb);
  }
  wave_sync();
  bool ok = sOk[wv];
  if (ok) {
    // lane (row, col) of the 8 x 8 DLT system: rows 2k, 2k+1 from correspondence k
    const int r = lane >> 3, c = lane & 7, k = r >> 1;
    const int2 p = sPts[wv][k], q = sPts[wv][4 + k];
    const double x = p.x, y = p.y, u2 = q.x, v2 = q.y;
    const double a = (r & 1) ? row1(c, x, y, v2) : row0(c, x, y, u2);
    double h = 0.0;
    ok = wave_solve8(a, (r & 1) ? v2 : u2, h);
    if (lane < 8) sH[wv][lane] = ok ? h : 0.0;
  } else if (lane < 8) {
    sH[wv][lane] = 0.0;
  }
  if (lane == 0) sH[wv][8] = 1.0;
  wave_sync();
  double H[9];
  for (int c = 0; c < 9; ++c) H[c] = sH[wv][c];
  int cnt = 0;
  if (ok)
    for (int k = lane; k < M; k += 64) cnt += is_inlier(H, qa[k], qb[k], eps2);
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if (lane == 0) {
    hyp_ok[t] = ok;
    hyp_counts[t] = ok ? cnt : 0;
  }
  if (lane < 9) hyp_h[(int64_t)t * 9 + lane] = H[lane];
}

__global__ void __launch_bounds__(256) k_prosac_hyp(const int32_t* __restrict__ misc, const int2* __restrict__ qa,
                                                    const int2* __restrict__ qb, const int64_t* __restrict__ tp,
                                                    int nhyp, const double* __restrict__ uniforms, double eps2,
                                                    double* __restrict__ hyp_h, int32_t* __restrict__ hyp_ok,
                                                    int32_t* __restrict__ hyp_counts) {
  prosac_hyp_body(misc, qa, qb, tp, nhyp, uniforms, eps2, hyp_h, hyp_ok, hyp_counts, blockIdx.x);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// block-wide sums (kWaves waves) of up to five values into every thread; sRed holds
// kWaves x 5 partials, added in a fixed order
template <int kWaves>
__device__ __forceinline__ void block_sums(double* sRed, double& a, double& b, double& c, double& d, double& e) {
  const int w = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  d = wave_sum(d);
  e = wave_sum(e);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sRed[w * 5 + 0] = a;
    sRed[w * 5 + 1] = b;
    sRed[w * 5 + 2] = c;
    sRed[w * 5 + 3] = d;
    sRed[w * 5 + 4] = e;
  }
  __syncthreads();
  a = b = c = d = e = 0.0;
  for (int k = 0; k < kWaves; ++k) {
    a += sRed[k * 5 + 0];
    b += sRed[k * 5 + 1];
    c += sRed[k * 5 + 2];
    d += sRed[k * 5 + 3];
    e += sRed[k * 5 + 4];
  }
}


constexpr int kFinalThreads = 512, kFinalWaves = kFinalThreads / 64;
constexpr int kParts = 7;                             // 72 x 7 = 504 of the 512 threads

// one block of kFinalThreads: the best hypothesis, its inliers, the least-squares refit
__device__ __forceinline__ void prosac_final_body(const int32_t* __restrict__ misc,
                                                  const int2* __restrict__ qa, const int2* __restrict__ qb,
                                                  const int32_t* __restrict__ qi, int cap_a, int nhyp,
                                                  const double* __restrict__ hyp_h,
                                                  const int32_t* __restrict__ hyp_ok,
                                                  const int32_t* __restrict__ hyp_counts, double eps2,
                                                  double* __restrict__ H_out, int32_t* __restrict__ inliers,
                                                  uint8_t* __restrict__ mask) {
  __shared__ unsigned long long sBest;
  __shared__ double sRed[kFinalWaves * 5];
  __shared__ double sPart[kParts][72];
  __shared__ double sH[9];
  __shared__ uint32_t sFlag[kMaxPoints / 32];
  const int tid = threadIdx.x;
  const int M = misc[0];
  if (tid == 0) sBest = 0ull;
  for (int i = tid; i < cap_a; i += kFinalThreads) mask[i] = 0;
  for (int i = tid; i < (M + 31) / 32; i += kFinalThreads) sFlag[i] = 0;
  __syncthreads();
  // best: most inliers, then the earliest hypothesis; key (count + 1) << 32 | (2^32-1 - t)
  unsigned long long mine = 0ull;
  for (int t = tid; t < nhyp; t += kFinalThreads)
    if (hyp_ok[t]) {
      const unsigned long long k = ((unsigned long long)(hyp_counts[t] + 1) << 32) | (0xFFFFFFFFull - (unsigned)t);
      mine = k > mine ? k : mine;
    }
  atomicMax(&sBest, mine);
  __syncthreads();
  const unsigned long long best = sBest;
  if (best == 0ull) {                                 // no valid hypothesis
    if (tid < 9) H_out[tid] = 0.0;
    if (tid == 0) *inliers = 0;
    return;
  }
  const int tb = (int)(0xFFFFFFFFull - (best & 0xFFFFFFFFull));
  if (tid < 9) sH[tid] = hyp_h[(int64_t)tb * 9 + tid];
  __syncthreads();
  double Hb[9];
  for (int c = 0; c < 9; ++c) Hb[c] = sH[c];
  // inliers of the best model (flags, mask over queries) and the sums for the normalisation
  double sx = 0, sy = 0, su = 0, sv = 0, cn = 0;
  for (int k = tid; k < M; k += kFinalThreads)
    if (is_inlier(Hb, qa[k], qb[k], eps2)) {
      atomicOr(&sFlag[k >> 5], 1u << (k & 31));
      mask[qi[k]] = 1;
      sx += qa[k].x;
      sy += qa[k].y;
      su += qb[k].x;
      sv += qb[k].y;
      cn += 1.0;
    }
  block_sums<kFinalWaves>(sRed, cn, sx, sy, su, sv);              // (its barriers also publish sFlag)
  const double n_in = cn;
  if (tid == 0) *inliers = (int)n_in;
  if (n_in < 5.0) {
    if (tid < 9) H_out[tid] = Hb[tid] / Hb[8];
    return;
  }
  const double cx = sx / n_in, cy = sy / n_in, cu = su / n_in, cv = sv / n_in;
  auto flag = [&](int k) { return (sFlag[k >> 5] >> (k & 31)) & 1u; };
  double da = 0, db = 0;
  for (int k = tid; k < M; k += kFinalThreads)
    if (flag(k)) {
      da += sqrt((qa[k].x - cx) * (qa[k].x - cx) + (qa[k].y - cy) * (qa[k].y - cy));
      db += sqrt((qb[k].x - cu) * (qb[k].x - cu) + (qb[k].y - cv) * (qb[k].y - cv));
    }
  double z0 = 0.0, z1 = 0.0, z2 = 0.0;
  block_sums<kFinalWaves>(sRed, da, db, z0, z1, z2);
  const double s_a = sqrt(2.0) / (da / n_in);
  const double s_b = sqrt(2.0) / (db / n_in);
  // normal equations of the normalised system: entry c (64 of A^T A, 8 of A^T b) summed by
  // kParts threads over interleaved inliers, then the parts in a fixed order
  if (tid < 72 * kParts) {
    const int c = tid % 72, part = tid / 72;
    const int a = c < 64 ? c / 8 : c - 64, cc = c % 8;
    double acc = 0.0;
    for (int k = part; k < M; k += kParts)
      if (flag(k)) {
        const double x = s_a * (qa[k].x - cx), y = s_a * (qa[k].y - cy);
        const double u = s_b * (qb[k].x - cu), v = s_b * (qb[k].y - cv);
        if (c < 64) acc += row0(a, x, y, u) * row0(cc, x, y, u) + row1(a, x, y, v) * row1(cc, x, y, v);
        else acc += row0(a, x, y, u) * u + row1(a, x, y, v) * v;
      }
    sPart[part][c] = acc;
  }
  __syncthreads();
  if (tid < 64) {                                     // wave 0 solves the normal equations
    const int r = tid >> 3;
    double a = 0.0, bv = 0.0;
    for (int k = 0; k < kParts; ++k) {
      a += sPart[k][tid];
      bv += sPart[k][64 + r];
    }
    double h = 0.0;
    const bool solved = wave_solve8(a, bv, h);
    if (tid < 8) sH[tid] = h;
    wave_sync();
    if (tid == 0 && solved) {
      double Hn[9];
      for (int c = 0; c < 8; ++c) Hn[c] = sH[c];
      Hn[8] = 1.0;
      // H = Tb^-1 Hn Ta with Ta = [s_a 0 -s_a cx; 0 s_a -s_a cy; 0 0 1], Tb likewise
      const double Ta[9] = {s_a, 0, -s_a * cx, 0, s_a, -s_a * cy, 0, 0, 1};
      const double Tbi[9] = {1.0 / s_b, 0, cu, 0, 1.0 / s_b, cv, 0, 0, 1};
      double HT[9], R[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double sum = 0.0;
          for (int k = 0; k < 3; ++k) sum += Hn[3 * r + k] * Ta[3 * k + c];
          HT[3 * r + c] = sum;
        }
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double sum = 0.0;
          for (int k = 0; k < 3; ++k) sum += Tbi[3 * r + k] * HT[3 * k + c];
          R[3 * r + c] = sum;
        }
      for (int c = 0; c < 9; ++c) H_out[c] = R[c] / R[8];
    } else if (tid == 0) {
      for (int c = 0; c < 9; ++c) H_out[c] = Hb[c] / Hb[8];
    }
  }
}

__global__ void __launch_bounds__(kFinalThreads) k_prosac_final(const int32_t* __restrict__ misc,
                                                       const int2* __restrict__ qa, const int2* __restrict__ qb,
                                                       const int32_t* __restrict__ qi, int cap_a, int nhyp,
                                                       const double* __restrict__ hyp_h,
                                                       const int32_t* __restrict__ hyp_ok,
                                                       const int32_t* __restrict__ hyp_counts, double eps2,
                                                       double* __restrict__ H_out, int32_t* __restrict__ inliers,
                                                       uint8_t* __restrict__ mask) {
  prosac_final_body(misc, qa, qb, qi, cap_a, nhyp, hyp_h, hyp_ok, hyp_counts, eps2, H_out, inliers, mask);
}

// Several pairs per launch of each PROSAC stage: blockIdx.y selects the pair and its
// descriptor (inputs, outputs and workspace region) from a device table.
struct ProsacPairDev {
  const int32_t* pts_a;
  const int32_t* pts_b;
  const int32_t* match;
  const int32_t* dist;
  const int32_t* count_a;
  const double* uniforms;
  int32_t* misc;
  int2* qa;
  int2* qb;
  int32_t* qi;
  int64_t* tp;
  double* hyp_h;
  int32_t* hyp_ok;
  int32_t* hyp_counts;
  double* H;
  int32_t* inliers;
  uint8_t* mask;
  int32_t cap_a, cap_b;
};

__global__ void __launch_bounds__(1024) k_prosac_prepare_multi(const ProsacPairDev* __restrict__ pairs,
                                                                const PairArgs<ProsacPairDev> args, double T_N) {
  const ProsacPairDev q = pair_of(pairs, args, blockIdx.y);
  prosac_prepare_body(q.pts_a, q.pts_b, q.cap_b, q.match, q.dist, q.count_a, q.cap_a, T_N, q.misc, q.qa, q.qb, q.qi,
                      q.tp);
}

__global__ void __launch_bounds__(256) k_prosac_hyp_multi(const ProsacPairDev* __restrict__ pairs,
                                                          const PairArgs<ProsacPairDev> args, int nhyp, double eps2) {
  const ProsacPairDev q = pair_of(pairs, args, blockIdx.y);
  prosac_hyp_body(q.misc, q.qa, q.qb, q.tp, nhyp, q.uniforms, eps2, q.hyp_h, q.hyp_ok, q.hyp_counts, blockIdx.x);
}

__global__ void __launch_bounds__(kFinalThreads) k_prosac_final_multi(const ProsacPairDev* __restrict__ pairs,
                                                                      const PairArgs<ProsacPairDev> args, int nhyp,
                                                                      double eps2) {
  const ProsacPairDev q = pair_of(pairs, args, blockIdx.y);
  prosac_final_body(q.misc, q.qa, q.qb, q.qi, q.cap_a, nhyp, q.hyp_h, q.hyp_ok, q.hyp_counts, eps2, q.H, q.inliers,
                    q.mask);
}

size_t up(size_t v) { return (v + 255) & ~(size_t)255; }

ProsacWs prosac_layout(int cap_a, int nhyp, size_t* total) {
  ProsacWs L;
  size_t o = 0;
  L.misc = o; o += 256;
  L.qa = o; o += up((size_t)cap_a * 8);
  L.qb = o; o += up((size_t)cap_a * 8);
  L.qi = o; o += up((size_t)cap_a * 4);
  L.tp = o; o += up((size_t)(cap_a + 1) * 8);
  L.hyp_h = o; o += up((size_t)nhyp * 9 * 8);
  L.hyp_ok = o; o += up((size_t)nhyp * 4);
  *total = o;
  return L;
}

}  // namespace

extern "C" {

size_t stitch_lsh_match_workspace_bytes(int32_t cap_a, int32_t cap_b, int32_t tables) {
  if (cap_a < 1 || cap_b < 1 || cap_a > kMaxPoints || cap_b > kMaxPoints || tables < 1 || tables > kMaxTables)
    return 0;
  return up((size_t)tables * cap_a * 4) + up((size_t)tables * cap_b * 4);
}

stitch_status stitch_lsh_match(int32_t nd, const uint32_t* desc_a, const int32_t* count_a, int32_t cap_a,
                               const uint32_t* desc_b, const int32_t* count_b, int32_t cap_b, int32_t tables,
                               int32_t kbits, const int32_t* positions, int32_t max_dist, int32_t* match,
                               int32_t* dist, void* workspace, size_t workspace_bytes, void* stream) {
  if (!desc_a || !count_a || !desc_b || !count_b || !match || !dist || (kbits > 0 && !positions))
    return fail(STITCH_E_NULL, "a descriptor, count, output or the positions is NULL");
  if (nd < 32 || nd > 512 || nd % 32) return fail(STITCH_E_SHAPE, "nd = %d is not a multiple of 32 in 32..512", nd);
  if (cap_a < 1 || cap_b < 1 || cap_a > kMaxPoints || cap_b > kMaxPoints)
    return fail(STITCH_E_SHAPE, "capacities must lie in 1..%d", kMaxPoints);
  if (tables < 1 || tables > kMaxTables || kbits < 0 || kbits > kMaxKeyBits)
    return fail(STITCH_E_SHAPE, "tables in 1..%d and key bits in 0..%d", kMaxTables, kMaxKeyBits);
  if ((uintptr_t)desc_a & 7 || (uintptr_t)desc_b & 7)
    return fail(STITCH_E_SHAPE, "descriptors must be 8-byte aligned");
  LshParams P{};
  P.tables = tables;
  P.kbits = kbits;
  P.words = nd / 32;
  for (int l = 0; l < tables; ++l)
    for (int b = 0; b < kbits; ++b) {
      const int p = positions[l * kbits + b];
      if (p < 0 || p >= nd) return fail(STITCH_E_SHAPE, "bit position %d outside 0..%d", p, nd - 1);
      P.pos[l][b] = (int16_t)p;
    }
  const size_t need = stitch_lsh_match_workspace_bytes(cap_a, cap_b, tables);
  if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 255))
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes", need);
  uint32_t* keys_a = (uint32_t*)workspace;
  uint32_t* keys_b = (uint32_t*)((uint8_t*)workspace + up((size_t)tables * cap_a * 4));
  const hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_lsh_keys, dim3((cap_a + 255) / 256), dim3(256), 0, s, desc_a, count_a, cap_a, P, keys_a);
  hipLaunchKernelGGL(k_lsh_keys, dim3((cap_b + 255) / 256), dim3(256), 0, s, desc_b, count_b, cap_b, P, keys_b);
  hipLaunchKernelGGL(k_lsh_match, dim3((cap_a + 3) / 4), dim3(256), 0, s, desc_a, count_a, cap_a, desc_b, count_b,
                     cap_b, P, keys_a, keys_b, max_dist, match, dist);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "matching launch");
  return STITCH_OK;
}

size_t stitch_lsh_match_multi_workspace_bytes(int32_t npairs, const stitch_match_pair* pairs, int32_t tables) {
  if (npairs < 1 || npairs > kMaxPairs || !pairs) return 0;
  size_t total = up((size_t)npairs * sizeof(LshPairDev));
  for (int p = 0; p < npairs; ++p) {
    const size_t one = stitch_lsh_match_workspace_bytes(pairs[p].cap_a, pairs[p].cap_b, tables);
    if (!one) return 0;
    total += one;
  }
  return total;
}

stitch_status stitch_lsh_match_multi(int32_t npairs, const stitch_match_pair* pairs, int32_t nd, int32_t tables,
                                     int32_t kbits, const int32_t* positions, int32_t max_dist, void* workspace,
                                     size_t workspace_bytes, void* stream) {
  if (!pairs || (kbits > 0 && !positions)) return fail(STITCH_E_NULL, "pairs or the positions is NULL");
  if (npairs < 1 || npairs > kMaxPairs) return fail(STITCH_E_SHAPE, "npairs = %d outside 1..%d", npairs, kMaxPairs);
  if (nd < 32 || nd > 512 || nd % 32) return fail(STITCH_E_SHAPE, "nd = %d is not a multiple of 32 in 32..512", nd);
  if (tables < 1 || tables > kMaxTables || kbits < 0 || kbits > kMaxKeyBits)
    return fail(STITCH_E_SHAPE, "tables in 1..%d and key bits in 0..%d", kMaxTables, kMaxKeyBits);
  LshParams P{};
  P.tables = tables;
  P.kbits = kbits;
  P.words = nd / 32;
  for (int l = 0; l < tables; ++l)
    for (int b = 0; b < kbits; ++b) {
      const int q = positions[l * kbits + b];
      if (q < 0 || q >= nd) return fail(STITCH_E_SHAPE, "bit position %d outside 0..%d", q, nd - 1);
      P.pos[l][b] = (int16_t)q;
    }
  for (int p = 0; p < npairs; ++p) {
    const stitch_match_pair& m = pairs[p];
    if (!m.desc_a || !m.count_a || !m.desc_b || !m.count_b || !m.match || !m.dist)
      return fail(STITCH_E_NULL, "pair %d: a descriptor, count or output is NULL", p);
    if (m.cap_a < 1 || m.cap_b < 1 || m.cap_a > kMaxPoints || m.cap_b > kMaxPoints)
      return fail(STITCH_E_SHAPE, "pair %d: capacities must lie in 1..%d", p, kMaxPoints);
    if ((uintptr_t)m.desc_a & 7 || (uintptr_t)m.desc_b & 7)
      return fail(STITCH_E_SHAPE, "pair %d: descriptors must be 8-byte aligned", p);
  }
  const size_t need = stitch_lsh_match_multi_workspace_bytes(npairs, pairs, tables);
  if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 255))
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes", need);
  int cap_max = 1, capa_max = 1;
  std::vector<LshPairDev> tab((size_t)npairs);
  uint8_t* ws = (uint8_t*)workspace;
  size_t o = up((size_t)npairs * sizeof(LshPairDev));
  for (int p = 0; p < npairs; ++p) {
    const stitch_match_pair& m = pairs[p];
    LshPairDev& d = tab[p];
    d.desc_a = m.desc_a; d.count_a = m.count_a; d.cap_a = m.cap_a;
    d.desc_b = m.desc_b; d.count_b = m.count_b; d.cap_b = m.cap_b;
    d.match = m.match; d.dist = m.dist;
    d.keys_a = (uint32_t*)(ws + o); o += up((size_t)tables * m.cap_a * 4);
    d.keys_b = (uint32_t*)(ws + o); o += up((size_t)tables * m.cap_b * 4);
    cap_max = std::max(cap_max, std::max(m.cap_a, m.cap_b));
    capa_max = std::max(capa_max, m.cap_a);
  }
  const hipStream_t s = (hipStream_t)stream;
  PairArgs<LshPairDev> args{};
  const LshPairDev* dev = nullptr;
  hipError_t e = hipSuccess;
  if (npairs <= kArgPairs) {
    for (int p = 0; p < npairs; ++p) args.p[p] = tab[p];
  } else {
    e = hipMemcpyAsync(workspace, tab.data(), tab.size() * sizeof(LshPairDev), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "matching table upload");
    dev = (const LshPairDev*)workspace;
  }
  hipLaunchKernelGGL(k_lsh_keys_multi, dim3((cap_max + 255) / 256, 2 * npairs), dim3(256), 0, s, dev, args, P);
  hipLaunchKernelGGL(k_lsh_match_multi, dim3((capa_max + 3) / 4, npairs), dim3(256), 0, s, dev, args, P, max_dist);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "matching launch");
  return STITCH_OK;
}

size_t stitch_prosac_workspace_bytes(int32_t cap_a, int32_t nhyp) {
  if (cap_a < 1 || cap_a > kMaxPoints || nhyp < 1 || nhyp > kMaxHyp) return 0;
  size_t total = 0;
  prosac_layout(cap_a, nhyp, &total);
  return total;
}

}  // extern "C"

namespace {

// Scratch of the allocation-free PROSAC entry point: one array per device that runs it,
// held until the process ends.  Host code never passes `scratch` itself to a kernel (on the
// host it only names the symbol); it passes the device address from hipGetSymbolAddress.
constexpr size_t kProsacScratchBytes = (size_t)1 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) uint8_t scratch[kProsacScratchBytes];
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of the scratch array (its address is looked up once per device,
// with that device current).
stitch_status prosac_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(STITCH_E_DEVICE, "device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return STITCH_OK;
}

stitch_status prosac_run(const int32_t* pts_a, const int32_t* pts_b, int32_t cap_b, const int32_t* match,
                         const int32_t* dist, const int32_t* count_a, int32_t cap_a, int32_t nhyp,
                         const double* uniforms, double T_N, double eps, double* H, int32_t* inliers,
                         uint8_t* inlier_mask, int32_t* hyp_counts, void* workspace, size_t workspace_bytes,
                         void* stream, bool own_scratch);

}  // namespace

extern "C" {

stitch_status stitch_prosac(const int32_t* pts_a, const int32_t* pts_b, int32_t cap_b, const int32_t* match,
                            const int32_t* dist, const int32_t* count_a, int32_t cap_a, int32_t nhyp,
                            const double* uniforms, double T_N, double eps, double* H, int32_t* inliers,
                            uint8_t* inlier_mask, int32_t* hyp_counts, void* workspace, size_t workspace_bytes,
                            void* stream) {
  return prosac_run(pts_a, pts_b, cap_b, match, dist, count_a, cap_a, nhyp, uniforms, T_N, eps, H, inliers,
                    inlier_mask, hyp_counts, workspace, workspace_bytes, stream, false);
}

stitch_status stitch_prosac_noalloc(const int32_t* pts_a, const int32_t* pts_b, int32_t cap_b, const int32_t* match,
                                    const int32_t* dist, const int32_t* count_a, int32_t cap_a, int32_t nhyp,
                                    const double* uniforms, double T_N, double eps, double* H, int32_t* inliers,
                                    uint8_t* inlier_mask, int32_t* hyp_counts, void* stream) {
  return prosac_run(pts_a, pts_b, cap_b, match, dist, count_a, cap_a, nhyp, uniforms, T_N, eps, H, inliers,
                    inlier_mask, hyp_counts, nullptr, 0, stream, true);
}

}  // extern "C"

namespace {

stitch_status prosac_run(const int32_t* pts_a, const int32_t* pts_b, int32_t cap_b, const int32_t* match,
                         const int32_t* dist, const int32_t* count_a, int32_t cap_a, int32_t nhyp,
                         const double* uniforms, double T_N, double eps, double* H, int32_t* inliers,
                         uint8_t* inlier_mask, int32_t* hyp_counts, void* workspace, size_t workspace_bytes,
                         void* stream, bool own_scratch) {
  if (!pts_a || !pts_b || !match || !dist || !count_a || !uniforms || !H || !inliers || !inlier_mask || !hyp_counts)
    return fail(STITCH_E_NULL, "an input or output is NULL");
  if (cap_a < 1 || cap_a > kMaxPoints || cap_b < 1 || cap_b > kMaxPoints)
    return fail(STITCH_E_SHAPE, "capacities must lie in 1..%d", kMaxPoints);
  if (nhyp < 1 || nhyp > kMaxHyp) return fail(STITCH_E_SHAPE, "nhyp = %d outside 1..%d", nhyp, kMaxHyp);
  if (!(T_N > 0.0) || !std::isfinite(T_N) || !(eps > 0.0) || !std::isfinite(eps))
    return fail(STITCH_E_SHAPE, "T_N and eps must be positive and finite");
  // the schedule T'_n grows to about T_N + M and is kept in int64: T_N up to 2^53 (where
  // every integer is still a double) leaves it far inside the range
  if (T_N > 0x1p53)
    return fail(STITCH_E_SHAPE, "T_N = %g exceeds 2^53", T_N);
  size_t need = 0;
  const ProsacWs L = prosac_layout(cap_a, nhyp, &need);
  if (own_scratch) {
    if (need > kProsacScratchBytes)
      return fail(STITCH_E_SHAPE, "cap_a = %d and nhyp = %d need %zu bytes of scratch; the allocation-free call "
                  "holds %zu", cap_a, nhyp, need, kProsacScratchBytes);
    const stitch_status st = prosac_scratch(&workspace);
    if (st) return st;
    workspace_bytes = kProsacScratchBytes;
  }
  if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 255))
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes", need);
  uint8_t* ws = (uint8_t*)workspace;
  int32_t* misc = (int32_t*)(ws + L.misc);
  int2* qa = (int2*)(ws + L.qa);
  int2* qb = (int2*)(ws + L.qb);
  int32_t* qi = (int32_t*)(ws + L.qi);
  int64_t* tp = (int64_t*)(ws + L.tp);
  double* hyp_h = (double*)(ws + L.hyp_h);
  int32_t* hyp_ok = (int32_t*)(ws + L.hyp_ok);
  const double eps2 = eps * eps;
  const hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_prosac_prepare, dim3(1), dim3(1024), 0, s, pts_a, pts_b, cap_b, match, dist, count_a, cap_a,
                     T_N, misc, qa, qb, qi, tp);
  hipLaunchKernelGGL(k_prosac_hyp, dim3((nhyp + 3) / 4), dim3(256), 0, s, misc, qa, qb, tp, nhyp, uniforms, eps2,
                     hyp_h, hyp_ok, hyp_counts);
  hipLaunchKernelGGL(k_prosac_final, dim3(1), dim3(kFinalThreads), 0, s, misc, qa, qb, qi, cap_a, nhyp, hyp_h, hyp_ok,
                     hyp_counts, eps2, H, inliers, inlier_mask);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "PROSAC launch");
  return STITCH_OK;
}

}  // namespace

namespace {

size_t prosac_multi_bytes(int32_t npairs, const stitch_prosac_pair* pairs, int32_t nhyp) {
  if (npairs < 1 || npairs > kMaxPairs || !pairs || nhyp < 1 || nhyp > kMaxHyp) return 0;
  size_t total = up((size_t)npairs * sizeof(ProsacPairDev));
  for (int p = 0; p < npairs; ++p) {
    if (pairs[p].cap_a < 1 || pairs[p].cap_a > kMaxPoints) return 0;
    size_t one = 0;
    prosac_layout(pairs[p].cap_a, nhyp, &one);
    total += one;
  }
  return total;
}

}  // namespace

extern "C" {

size_t stitch_prosac_multi_workspace_bytes(int32_t npairs, const stitch_prosac_pair* pairs, int32_t nhyp) {
  return prosac_multi_bytes(npairs, pairs, nhyp);
}

stitch_status stitch_prosac_multi(int32_t npairs, const stitch_prosac_pair* pairs, int32_t nhyp, double T_N,
                                  double eps, void* workspace, size_t workspace_bytes, void* stream) {
  if (!pairs) return fail(STITCH_E_NULL, "pairs is NULL");
  if (npairs < 1 || npairs > kMaxPairs) return fail(STITCH_E_SHAPE, "npairs = %d outside 1..%d", npairs, kMaxPairs);
  if (nhyp < 1 || nhyp > kMaxHyp) return fail(STITCH_E_SHAPE, "nhyp = %d outside 1..%d", nhyp, kMaxHyp);
  if (!(T_N > 0.0) || !std::isfinite(T_N) || !(eps > 0.0) || !std::isfinite(eps))
    return fail(STITCH_E_SHAPE, "T_N and eps must be positive and finite");
  if (T_N > 0x1p53) return fail(STITCH_E_SHAPE, "T_N = %g exceeds 2^53", T_N);
  for (int p = 0; p < npairs; ++p) {
    const stitch_prosac_pair& m = pairs[p];
    if (!m.pts_a || !m.pts_b || !m.match || !m.dist || !m.count_a || !m.uniforms || !m.H || !m.inliers ||
        !m.inlier_mask || !m.hyp_counts)
      return fail(STITCH_E_NULL, "pair %d: an input or output is NULL", p);
    if (m.cap_a < 1 || m.cap_a > kMaxPoints || m.cap_b < 1 || m.cap_b > kMaxPoints)
      return fail(STITCH_E_SHAPE, "pair %d: capacities must lie in 1..%d", p, kMaxPoints);
  }
  const size_t need = prosac_multi_bytes(npairs, pairs, nhyp);
  if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 255))
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes", need);
  std::vector<ProsacPairDev> tab((size_t)npairs);
  uint8_t* ws = (uint8_t*)workspace;
  size_t o = up((size_t)npairs * sizeof(ProsacPairDev));
  for (int p = 0; p < npairs; ++p) {
    const stitch_prosac_pair& m = pairs[p];
    size_t one = 0;
    const ProsacWs L = prosac_layout(m.cap_a, nhyp, &one);
    ProsacPairDev& d = tab[p];
    d.pts_a = m.pts_a; d.pts_b = m.pts_b; d.match = m.match; d.dist = m.dist; d.count_a = m.count_a;
    d.uniforms = m.uniforms; d.cap_a = m.cap_a; d.cap_b = m.cap_b;
    d.misc = (int32_t*)(ws + o + L.misc);
    d.qa = (int2*)(ws + o + L.qa);
    d.qb = (int2*)(ws + o + L.qb);
    d.qi = (int32_t*)(ws + o + L.qi);
    d.tp = (int64_t*)(ws + o + L.tp);
    d.hyp_h = (double*)(ws + o + L.hyp_h);
    d.hyp_ok = (int32_t*)(ws + o + L.hyp_ok);
    d.hyp_counts = m.hyp_counts; d.H = m.H; d.inliers = m.inliers; d.mask = m.inlier_mask;
    o += one;
  }
  const double eps2 = eps * eps;
  const hipStream_t s = (hipStream_t)stream;
  PairArgs<ProsacPairDev> args{};
  const ProsacPairDev* dev = nullptr;
  hipError_t e = hipSuccess;
  if (npairs <= kArgPairs) {
    for (int p = 0; p < npairs; ++p) args.p[p] = tab[p];
  } else {
    e = hipMemcpyAsync(workspace, tab.data(), tab.size() * sizeof(ProsacPairDev), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "PROSAC table upload");
    dev = (const ProsacPairDev*)workspace;
  }
  hipLaunchKernelGGL(k_prosac_prepare_multi, dim3(1, npairs), dim3(1024), 0, s, dev, args, T_N);
  hipLaunchKernelGGL(k_prosac_hyp_multi, dim3((nhyp + 3) / 4, npairs), dim3(256), 0, s, dev, args, nhyp, eps2);
  hipLaunchKernelGGL(k_prosac_final_multi, dim3(1, npairs), dim3(kFinalThreads), 0, s, dev, args, nhyp, eps2);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "PROSAC launch");
  return STITCH_OK;
}

}  // extern "C"
