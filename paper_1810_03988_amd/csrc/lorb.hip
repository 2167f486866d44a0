// L-ORB feature extraction on gfx950 (Sec. 4.1, Alg. 1 and Alg. 2): in each feature
// detection area of a frame, FAST corners scored by the Harris response, non-maximal
// suppression, the N strongest, and their BRIEF descriptors.  All decisions are exact
// integer arithmetic:
//   gray level      g = (77 R + 150 G + 29 B + 128) >> 8
//   FAST            >= 9 contiguous pixels of the radius-3 circle brighter than g + tf or
//                   darker than g - tf
//   Harris          central-difference gradients, 5x5 binomial window b b^T (sigma = 1),
//                   R = 64 (A B - C^2) - 3 (A + B)^2  (alpha = 3/64, scaled by 64), int64
//   candidates      FAST corners with R >= t; suppression over 3x3 among candidates, ties
//                   to the first in raster order; the N of largest R, ties by raster order
//   BRIEF           three-valued tests of n_d point pairs on S = b b^T * g (integer sums),
//                   kept as a "greater" and a "less" bit string
// Points must keep their descriptor support in the frame (17 samples from every edge);
// areas are clipped to that range.
//
// Five launches per call, each covering every area of every frame of the call:
//   k_lorb_clear    zero the areas' survivor counts
//   k_lorb_detect   64x16 tiles: gray tile with a 4-sample halo in LDS, the horizontal pass
//                   of the window over the gradient products (formed on the fly) in LDS,
//                   the vertical pass, the FAST test and R on the tile plus a 1-sample
//                   ring, suppression from LDS; survivors are appended to the area's list
//                   (one atomic per block; list order is arbitrary)
//   k_lorb_select   one block per area: a histogram of the survivors over a monotone bucket
//                   of R in LDS, the highest bucket b such that the buckets >= b hold at
//                   least N survivors (all buckets when there are fewer), and the survivors
//                   in buckets >= b copied to a short list.  Every survivor that precedes
//                   one of them in the order below is among them, so their ranks in the
//                   short list are their ranks among all survivors.
//   k_lorb_rank     rank of each short-list entry in the total order (R descending, raster
//                   index ascending): the four waves of a block count, for the same 64
//                   entries, the preceding entries in a quarter of the short list each,
//                   read with uniform (scalar) loads; ranks below N go to the outputs
//   k_lorb_brief    one wave per kept point: its 35x35 gray patch and the horizontal pass
//                   of the window in LDS, the vertical pass per tested sample
// Because the order is total, the result does not depend on the list order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <mutex>
#include <vector>

#include "stitch_internal.h"

using namespace stitch;

namespace {

constexpr int kMargin = 17;
constexpr int kMaxAreas = 64;
constexpr int kTX = 64, kTY = 16;                       // outputs per tile
constexpr int kGW = kTX + 8, kGH = kTY + 8;             // gray: tile + 4 each side (72 x 24)
constexpr int kPH = kTY + 6;                            // gradient-product rows: tile + 3 (22)
constexpr int kHW = kTX + 2;                            // horizontal pass: tile + 1 (66 x 22)
constexpr int kRW = kTX + 2, kRH = kTY + 2;             // responses: tile + 1 (66 x 18)
constexpr int kBins = 4096;                             // response histogram per area
constexpr int kRankGrid = 64;
constexpr int kPatch = 35, kHalfPatch = 17;             // gray patch of a point (15 + 2)
constexpr int64_t kNone = INT64_MIN;

constexpr int kMaxFrames = 16;

struct AreaDesc {
  int32_t x0, y0, w, h;        // clipped area (frame coordinates)
  int32_t tiles_x, ntiles, tile_begin, list_off;
  int32_t frame;               // index into AreaTable::f
};

struct FrameRef {
  const uint8_t* p;            // U8 HWC RGB
  int64_t row;                 // bytes
  int32_t w, h;
};

struct AreaTable {
  int32_t m, n_max, nd, pad;
  AreaDesc a[kMaxAreas];
  FrameRef f[kMaxFrames];
};

__device__ __forceinline__ int luma3(uint32_t r, uint32_t g, uint32_t b) {
  return (int)((77 * r + 150 * g + 29 * b + 128) >> 8);
}

// Bytes at any address (global memory accepts unaligned dword accesses).
#define GLB __attribute__((address_space(1)))
typedef unsigned long long __attribute__((aligned(1))) u64u;
typedef uint32_t __attribute__((aligned(1))) u32u;
__device__ __forceinline__ unsigned long long ld8u(const uint8_t* p) { return *(const GLB u64u*)p; }
__device__ __forceinline__ uint32_t ld4u(const uint8_t* p) { return *(const GLB u32u*)p; }

// gray levels of the 4 RGB pixels in the 12 bytes at p
__device__ __forceinline__ int4 luma4(const uint8_t* p) {
  const unsigned long long lo = ld8u(p);
  const uint32_t hi = ld4u(p + 8);
  auto B = [&](int i) -> uint32_t { return i < 8 ? (uint32_t)(lo >> (8 * i)) & 255u : (hi >> (8 * (i - 8))) & 255u; };
  return make_int4(luma3(B(0), B(1), B(2)), luma3(B(3), B(4), B(5)), luma3(B(6), B(7), B(8)),
                   luma3(B(9), B(10), B(11)));
}

// FAST circle of radius 3, clockwise from the top
__constant__ int8_t kCircle[16][2] = {{0, -3}, {1, -3}, {2, -2}, {3, -1}, {3, 0}, {3, 1}, {2, 2}, {1, 3},
                                      {0, 3}, {-1, 3}, {-2, 2}, {-3, 1}, {-3, 0}, {-3, -1}, {-2, -2}, {-1, -3}};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Monotone (non-decreasing) bucket of a response: zero in the middle, then by binary
// exponent and the next five bits of |R| on either side (like the leading bits of a
// floating-point number).  R is never INT64_MIN.
__device__ __forceinline__ int bucket(int64_t R) {
  if (R == 0) return kBins / 2;
  const uint64_t v = R > 0 ? (uint64_t)R : (uint64_t)(-R);
  const int e = 63 - __clzll(v);
  const int m5 = (e >= 5 ? (int)(v >> (e - 5)) : (int)(v << (5 - e))) & 31;
  const int k = min(e * 32 + m5, kBins / 2 - 2);
  return R > 0 ? kBins / 2 + 1 + k : kBins / 2 - 1 - k;
}

__global__ void k_lorb_clear(int32_t* __restrict__ count, int m) {
  if ((int)threadIdx.x < 2 * m) count[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256) k_lorb_detect(const AreaTable T, int tf, int64_t t,
                                                     int32_t* __restrict__ count, int64_t* __restrict__ listR,
                                                     int32_t* __restrict__ listI) {
  __shared__ __attribute__((aligned(16))) int sG[kGH][kGW + 4];
  __shared__ int sWave[4];
  __shared__ int sBase;
  __shared__ int sH[3][kPH][kHW];
  __shared__ int64_t sR[kRH][kRW];                   // responses, kNone where no candidate
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  int z = 0;
  for (int i = 0; i < T.m; ++i)
    if (b >= T.a[i].tile_begin && b < T.a[i].tile_begin + T.a[i].ntiles) z = i;
  const AreaDesc a = T.a[z];
  const uint8_t* __restrict__ frame = T.f[a.frame].p;
  const int64_t row = T.f[a.frame].row;
  const int fw = T.f[a.frame].w, fh = T.f[a.frame].h;
  const int tl = b - a.tile_begin;
  const int ty = tl / a.tiles_x, tx = tl - ty * a.tiles_x;
  const int ox = tx * kTX, oy = ty * kTY;                    // tile origin (area coordinates)
  // gray levels on area columns ox-4 .. ox+67, rows oy-4 .. oy+19, four pixels (12 bytes)
  // per load.  Rows past the frame repeat its last row and groups reaching past its right
  // edge start at its last four pixels: positions of the area need gray levels at most 3
  // samples beyond it, which lie 14 or more inside the frame, so such groups and rows only
  // feed positions outside the area, which are never candidates.
  {
    const int xs = a.x0 + ox - 4, ys = a.y0 + oy - 4;
    for (int e = tid; e < kGH * (kGW / 4); e += 256) {
      const int r = e / (kGW / 4), g = e - r * (kGW / 4);
      const int x = min(xs + 4 * g, fw - 4), y = min(ys + r, fh - 1);
      *reinterpret_cast<int4*>(&sG[r][4 * g]) = luma4(frame + (int64_t)y * row + 3 * (int64_t)x);
    }
  }
  __syncthreads();
  // gradient products (on columns ox-3 .. ox+66, rows oy-3 .. oy+18) and the binomial
  // window [1 4 6 4 1] horizontally (columns ox-1 .. ox+64): each output forms the gradients
  // of its five taps from the gray levels and weights their three products
  for (int e = tid; e < kPH * kHW; e += 256) {
    const int r = e / kHW, c = e - r * kHW;
    int pxx[5], pyy[5], pxy[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {                  // product column c + i (gray column c + i + 1)
      const int ix = sG[r + 1][c + i + 2] - sG[r + 1][c + i], iy = sG[r + 2][c + i + 1] - sG[r][c + i + 1];
      pxx[i] = ix * ix;
      pyy[i] = iy * iy;
      pxy[i] = ix * iy;
    }
    sH[0][r][c] = (pxx[0] + pxx[4]) + 4 * (pxx[1] + pxx[3]) + 6 * pxx[2];
    sH[1][r][c] = (pyy[0] + pyy[4]) + 4 * (pyy[1] + pyy[3]) + 6 * pyy[2];
    sH[2][r][c] = (pxy[0] + pxy[4]) + 4 * (pxy[1] + pxy[3]) + 6 * pxy[2];
  }
  __syncthreads();
  // vertically, the response and the segment test on the tile and a 1-sample ring
  // (kRH * kRW = 1188 positions: at most 5 per thread)
  int64_t resp[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int e = tid + 256 * k;
    int64_t out = kNone;
    if (e < kRH * kRW) {
      const int r = e / kRW, c = e - r * kRW;
      const int ax = ox - 1 + c, ay = oy - 1 + r;
      if (ax >= 0 && ax < a.w && ay >= 0 && ay < a.h) {
        const int gr = r + 3, gc = c + 3;
        const int p = sG[gr][gc];
        unsigned bright = 0, dark = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int v = sG[gr + kCircle[q][1]][gc + kCircle[q][0]];
          bright |= (unsigned)(v > p + tf) << q;
          dark |= (unsigned)(v < p - tf) << q;
        }
        // 9 contiguous set bits on the cyclic circle: bit i survives the shifts when bits
        // i .. i+8 of the doubled mask are all set
        unsigned mb = bright | (bright << 16), md = dark | (dark << 16);
#pragma unroll
        for (int s = 1; s < 9; ++s) {
          mb &= mb >> 1;
          md &= md >> 1;
        }
        if (((mb | md) & 0xFFFFu) != 0) {
          int64_t mm[3];
#pragma unroll
          for (int q = 0; q < 3; ++q)
            mm[q] = (int64_t)(sH[q][r][c] + sH[q][r + 4][c]) + 4 * (int64_t)(sH[q][r + 1][c] + sH[q][r + 3][c]) +
                    6 * (int64_t)sH[q][r + 2][c];
          const int64_t A = mm[0], B = mm[1], C = mm[2];
          const int64_t R = 64 * (A * B - C * C) - 3 * (A + B) * (A + B);
          if (R >= t) out = R;
        }
      }
    }
    resp[k] = out;
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int e = tid + 256 * k;
    if (e < kRH * kRW) sR[e / kRW][e % kRW] = resp[k];
  }
  __syncthreads();
  // suppression on the tile: a candidate survives when every neighbouring candidate has a
  // smaller R, or an equal R and a later raster position
  const int lane = tid & 63, wave = tid >> 6;
  constexpr int kPer = kTX * kTY / 256;              // 4 positions per thread
  int64_t keepR[kPer];
  uint64_t mask[kPer];
  int nwave = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int e = tid + 256 * k;
    const int r = e / kTX, c = e - r * kTX;
    const int64_t R = sR[r + 1][c + 1];
    bool keep = R != kNone;
    if (keep) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy) continue;
          const int64_t q = sR[r + 1 + dy][c + 1 + dx];
          const bool earlier = dy < 0 || (dy == 0 && dx < 0);
          if (q != kNone && (q > R || (q == R && earlier))) keep = false;
        }
    }
    keepR[k] = keep ? R : kNone;
    mask[k] = __ballot(keep);
    nwave += __popcll(mask[k]);
  }
  // append the block's survivors to the area's list with one atomic
  if (lane == 0) sWave[wave] = nwave;
  __syncthreads();
  if (tid == 0) {
    const int total = sWave[0] + sWave[1] + sWave[2] + sWave[3];
    sBase = total ? atomicAdd(&count[2 * z], total) : 0;
  }
  __syncthreads();
  int run = sBase;
  for (int w = 0; w < wave; ++w) run += sWave[w];
  const uint64_t below = (1ull << lane) - 1;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (keepR[k] != kNone) {
      const int e = tid + 256 * k;
      const int r = e / kTX, c = e - r * kTX;
      const int pos = a.list_off + run + __popcll(mask[k] & below);
      listR[pos] = keepR[k];
      listI[pos] = (oy + r) * a.w + (ox + c);
    }
    run += __popcll(mask[k]);
  }
}

// grid m, 1024 threads: block z histograms area z's survivors, finds the threshold bucket
// and copies the survivors at or above it to the short list (padded to a multiple of 16
// with entries that precede nothing); writes the short-list length and counts[z].  The
// list is read eight entries per thread at a time.
__global__ void __launch_bounds__(1024) k_lorb_select(const AreaTable T, int32_t* __restrict__ count,
                                                      const int64_t* __restrict__ listR,
                                                      const int32_t* __restrict__ listI,
                                                      int64_t* __restrict__ shortR, int32_t* __restrict__ shortI,
                                                      int32_t* __restrict__ counts) {
  constexpr int kT = 1024, kU = 8, kPerT = kBins / kT;   // 4 consecutive bins per thread
  __shared__ int sHist[kBins];
  __shared__ int sSum[kT];
  __shared__ int sB, sCnt;
  const int z = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int c = count[2 * z], N = T.n_max, off = T.a[z].list_off;
  for (int q = tid; q < kBins; q += kT) sHist[q] = 0;
  if (tid == 0) {
    sB = 0;                                          // fewer than N survivors: every bucket
    sCnt = 0;
  }
  __syncthreads();
  if (c > N) {
    for (int base = 0; base < c; base += kT * kU) {
      int64_t R[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = base + u * kT + tid;
        R[u] = i < c ? listR[off + i] : kNone;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (R[u] != kNone) atomicAdd(&sHist[bucket(R[u])], 1);
    }
    __syncthreads();
    int local = 0;
#pragma unroll
    for (int q = 0; q < kPerT; ++q) local += sHist[kPerT * tid + q];
    sSum[tid] = local;
    __syncthreads();
    // inclusive suffix sums over the threads' totals (Hillis-Steele)
    for (int d = 1; d < kT; d <<= 1) {
      const int v = tid + d < kT ? sSum[tid + d] : 0;
      __syncthreads();
      sSum[tid] += v;
      __syncthreads();
    }
    const int above = sSum[tid] - local;             // survivors in higher threads' bins
    if (above < N && sSum[tid] >= N) {
      int acc = above, b = kPerT * tid;
      for (int q = kPerT - 1; q >= 0; --q) {
        acc += sHist[kPerT * tid + q];
        if (acc >= N) {
          b = kPerT * tid + q;
          break;
        }
      }
      sB = b;
    }
    __syncthreads();
  }
  const int bstar = sB;
  for (int base = 0; base < c; base += kT * kU) {   // the same trip count for every thread
    int64_t R[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = base + u * kT + tid;
      R[u] = i < c ? listR[off + i] : kNone;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool keep = R[u] != kNone && bucket(R[u]) >= bstar;
      const uint64_t mask = __ballot(keep);
      if (mask) {
        const int first = __ffsll((unsigned long long)mask) - 1;
        int wbase = 0;
        if (lane == first) wbase = atomicAdd(&sCnt, __popcll(mask));
        wbase = __shfl(wbase, first);
        if (keep) {
          const int pos = off + wbase + __popcll(mask & ((1ull << lane) - 1));
          shortR[pos] = R[u];
          shortI[pos] = listI[off + base + u * kT + tid];
        }
      }
    }
  }
  __syncthreads();
  // pad the short list to a multiple of 16 with entries that precede nothing
  const int cs = sCnt;
  if (tid < ((cs + 15) & ~15) - cs) {
    shortR[off + cs + tid] = kNone;
    shortI[off + cs + tid] = INT32_MAX;
  }
  if (tid == 0) {
    count[2 * z + 1] = cs;
    counts[z] = min(c, N);
  }
}

// grid (kRankGrid, m): the rank of short-list entry i of area z is the number of entries that
// precede it (R descending, raster index ascending); entries of rank < N go to output slot
// rank.  A block takes 64 entries; each of its waves counts over a quarter of the (padded)
// short list, sixteen entries per step with uniform loads.
__global__ void __launch_bounds__(256) k_lorb_rank(const AreaTable T, const int32_t* __restrict__ count,
                                                   const int64_t* __restrict__ shortR,
                                                   const int32_t* __restrict__ shortI, int32_t* __restrict__ pts,
                                                   int64_t* __restrict__ resp) {
  __shared__ int sPart[4][64];
  const int z = blockIdx.y, lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const AreaDesc& a = T.a[z];
  const int cs = count[2 * z + 1], N = T.n_max, off = a.list_off;
  const int cpad = (cs + 15) & ~15;
  const int span = ((cpad / 16 + 3) / 4) * 16;        // entries per wave, a multiple of 16
  const int j0 = min(cpad, wv * span), j1 = min(cpad, j0 + span);
  for (int item = blockIdx.x; item * 64 < cs; item += gridDim.x) {
    const int i = item * 64 + lane;
    const int ii = min(i, cs - 1);
    const int64_t Ri = shortR[off + ii];
    const int32_t Ii = shortI[off + ii];
    int cnt = 0;
    for (int j = j0; j < j1; j += 16) {
      int64_t Rj[16];
      int32_t Ij[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        Rj[q] = shortR[off + j + q];
        Ij[q] = shortI[off + j + q];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) cnt += (Rj[q] > Ri) | ((Rj[q] == Ri) & (Ij[q] < Ii));
    }
    sPart[wv][lane] = cnt;
    __syncthreads();
    if (wv == 0) {
      const int rk = sPart[0][lane] + sPart[1][lane] + sPart[2][lane] + sPart[3][lane];
      if (i < cs && rk < N) {
        const int y = Ii / a.w, x = Ii - y * a.w;
        const int64_t slot = (int64_t)z * N + rk;
        pts[2 * slot] = a.x0 + x;
        pts[2 * slot + 1] = a.y0 + y;
        resp[slot] = Ri;
      }
    }
    __syncthreads();
  }
}

// One wave per kept point: the 35x35 gray patch around it and the horizontal pass of the
// window in the wave's LDS; each tested sample takes the vertical pass from there.  Pattern
// offsets are clamped to +-15 so that every read stays in the patch.
__global__ void __launch_bounds__(256) k_lorb_brief(const AreaTable T,
                                                    const int32_t* __restrict__ pattern,
                                                    const int32_t* __restrict__ counts,
                                                    const int32_t* __restrict__ pts, uint32_t* __restrict__ desc) {
  __shared__ __attribute__((aligned(16))) int sPG[4][kPatch][kPatch + 1];
  __shared__ int sPH[4][kPatch][31];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int z = blockIdx.y, n_max = T.n_max, nd = T.nd;
  const int k = blockIdx.x * 4 + wv;
  if (k >= counts[z]) return;                        // whole waves leave; no block barrier below
  const int64_t slot = (int64_t)z * n_max + k;
  const int x = pts[2 * slot], y = pts[2 * slot + 1];
  const uint8_t* __restrict__ frame = T.f[T.a[z].frame].p;
  const int64_t row = T.f[T.a[z].frame].row;
  const uint8_t* base = frame + (int64_t)(y - kHalfPatch) * row + 3 * (int64_t)(x - kHalfPatch);
  // per row: 8 groups of 4 pixels (12 bytes) and a tail of 3 pixels (9 bytes); every byte
  // read belongs to the patch, which lies inside the frame
  for (int e = lane; e < kPatch * 9; e += 64) {
    const int r = e / 9, g = e - r * 9;
    const uint8_t* p = base + (int64_t)r * row + 12 * g;
    if (g < 8) {
      *reinterpret_cast<int4*>(&sPG[wv][r][4 * g]) = luma4(p);
    } else {
      const unsigned long long lo = ld8u(p);
      const uint32_t b8 = p[8];
      sPG[wv][r][32] = luma3((uint32_t)lo & 255u, (uint32_t)(lo >> 8) & 255u, (uint32_t)(lo >> 16) & 255u);
      sPG[wv][r][33] = luma3((uint32_t)(lo >> 24) & 255u, (uint32_t)(lo >> 32) & 255u, (uint32_t)(lo >> 40) & 255u);
      sPG[wv][r][34] = luma3((uint32_t)(lo >> 48) & 255u, (uint32_t)(lo >> 56) & 255u, b8);
    }
  }
  wave_sync_lds();
  for (int e = lane; e < kPatch * 31; e += 64) {
    const int r = e / 31, c = e - r * 31;
    const int* g = &sPG[wv][r][c];
    sPH[wv][r][c] = (g[0] + g[4]) + 4 * (g[1] + g[3]) + 6 * g[2];
  }
  wave_sync_lds();
  auto S = [&](int dx, int dy) {           // S at offset (dx, dy), both in -15 .. 15
    const int c = dx + 15, r = dy + 15;
    return (sPH[wv][r][c] + sPH[wv][r + 4][c]) + 4 * (sPH[wv][r + 1][c] + sPH[wv][r + 3][c]) +
           6 * sPH[wv][r + 2][c];
  };
  auto off = [](int32_t v) { return min(max(v, -15), 15); };
  const int words = nd / 32;
  uint32_t* d = desc + slot * 2 * words;
  for (int b0 = 0; b0 < nd; b0 += 64) {
    const int pk = b0 + lane;
    bool gt = false, lt = false;
    if (pk < nd) {
      const int4 pp = *reinterpret_cast<const int4*>(pattern + 4 * pk);
      const int s1 = S(off(pp.x), off(pp.y)), s2 = S(off(pp.z), off(pp.w));
      gt = s1 > s2;
      lt = s1 < s2;
    }
    const uint64_t mg = __ballot(gt), ml = __ballot(lt);
    const int w0 = b0 / 32;
    // lanes 0-3 store the (up to) two words of each string
    if (lane < 4) {
      const int hi = lane & 1, str = lane >> 1;
      if (w0 + hi < words) {
        const uint64_t mk = str ? ml : mg;
        d[str * words + w0 + hi] = (uint32_t)(hi ? (mk >> 32) : mk);
      }
    }
  }
}

AreaDesc clip(const int32_t* r, int fw, int fh) {
  AreaDesc a{};
  const int64_t x1 = std::min<int64_t>((int64_t)r[0] + r[2], fw - kMargin);
  const int64_t y1 = std::min<int64_t>((int64_t)r[1] + r[3], fh - kMargin);
  a.x0 = std::max(r[0], kMargin);
  a.y0 = std::max(r[1], kMargin);
  a.w = (int32_t)std::max<int64_t>(0, x1 - a.x0);
  a.h = (int32_t)std::max<int64_t>(0, y1 - a.y0);
  if (a.w == 0 || a.h == 0) a.w = a.h = 0;
  return a;
}

size_t up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
  int64_t total = 0;           // list entries (samples of all clipped areas, padded)
  size_t count = 0, listR = 0, listI = 0, shortR = 0, shortI = 0, bytes = 0;
};

// Area table and workspace layout for the areas of nframes frames (m_per_frame[f] areas of
// frame f, consecutive in areas); false when they are too large for 32-bit indices
bool plan_areas(int nframes, const int32_t* fw, const int32_t* fh, const int32_t* m_per_frame,
                const int32_t* areas, AreaTable& T, Layout& L) {
  int m = 0;
  for (int f = 0; f < nframes; ++f) m += m_per_frame[f];
  T.m = m;
  int64_t tiles = 0, total = 0;
  int frame = 0, left = m_per_frame[0];
  for (int i = 0; i < m; ++i) {
    while (left == 0) left = m_per_frame[++frame];
    --left;
    AreaDesc a = clip(areas + 4 * i, fw[frame], fh[frame]);
    a.frame = frame;
    a.tiles_x = (a.w + kTX - 1) / kTX;
    a.ntiles = a.tiles_x * ((a.h + kTY - 1) / kTY);
    a.tile_begin = (int32_t)tiles;
    a.list_off = (int32_t)total;                     // a multiple of 16
    tiles += a.ntiles;
    total += (((int64_t)a.w * a.h + 15) & ~(int64_t)15) + 16;   // room for the padding
    T.a[i] = a;
    if (total >= ((int64_t)1 << 30)) return false;
  }
  L.total = total;
  size_t o = 0;
  L.count = o; o += up((size_t)m * 2 * 4);
  L.listR = o; o += up((size_t)total * 8);
  L.listI = o; o += up((size_t)total * 4);
  L.shortR = o; o += up((size_t)total * 8);
  L.shortI = o; o += up((size_t)total * 4);
  L.bytes = o;
  return true;
}

// Per-launch event timing of stitch_lorb (diagnostics), process-wide.  While enabled, a
// call records an event before its first launch and one after each launch.
constexpr int kKinds = 5;                  // clear, detect, select, rank, brief
struct LorbTiming {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> spare;
  std::vector<std::array<hipEvent_t, kKinds + 1>> done;
  double ms[kKinds] = {};
  int32_t n[kKinds] = {};
  void recycle() {
    for (auto& c : done)
      for (hipEvent_t e : c) spare.push_back(e);
    done.clear();
  }
};
LorbTiming& timing() {
  static LorbTiming* t = new LorbTiming;   // never destroyed: events outlive static teardown
  return *t;
}

stitch_status check_areas(int32_t nframes, const int32_t* frame_w, const int32_t* frame_h,
                          const int32_t* m_per_frame, const int32_t* areas) {
  if (nframes < 1 || nframes > kMaxFrames) return fail(STITCH_E_SHAPE, "%d frames outside 1..%d", nframes, kMaxFrames);
  if (!frame_w || !frame_h || !m_per_frame || !areas) return fail(STITCH_E_NULL, "sizes, counts or areas is NULL");
  int m = 0;
  for (int f = 0; f < nframes; ++f) {
    if (m_per_frame[f] < 0 || m_per_frame[f] > kMaxAreas) return fail(STITCH_E_SHAPE, "frame %d: bad area count", f);
    m += m_per_frame[f];
    if (frame_w[f] < 2 * kMargin + 1 || frame_h[f] < 2 * kMargin + 1)
      return fail(STITCH_E_SHAPE, "frames need at least %d samples per side", 2 * kMargin + 1);
  }
  if (m < 1 || m > kMaxAreas) return fail(STITCH_E_SHAPE, "m = %d areas outside 1..%d", m, kMaxAreas);
  for (int i = 0; i < m; ++i)
    if (areas[4 * i + 2] < 0 || areas[4 * i + 3] < 0) return fail(STITCH_E_SHAPE, "area %d has a negative size", i);
  return STITCH_OK;
}

stitch_status lorb_run(int32_t nframes, const stitch_image* frames, const int32_t* m_per_frame,
                       const int32_t* areas, int32_t fast_threshold, int64_t harris_threshold, int32_t n_max,
                       int32_t nd, const int32_t* pattern, int32_t* counts, int32_t* points, int64_t* responses,
                       uint32_t* descriptors, void* workspace, size_t workspace_bytes, void* stream);

}  // namespace

extern "C" {

size_t stitch_lorb_multi_workspace_bytes(int32_t nframes, const int32_t* frame_w, const int32_t* frame_h,
                                         const int32_t* m_per_frame, const int32_t* areas) {
  if (check_areas(nframes, frame_w, frame_h, m_per_frame, areas)) return 0;
  AreaTable T;
  Layout L;
  if (!plan_areas(nframes, frame_w, frame_h, m_per_frame, areas, T, L)) {
    fail(STITCH_E_SHAPE, "the areas hold 2^30 samples or more");
    return 0;
  }
  return L.bytes;
}

size_t stitch_lorb_workspace_bytes(int32_t frame_w, int32_t frame_h, int32_t m, const int32_t* areas) {
  return stitch_lorb_multi_workspace_bytes(1, &frame_w, &frame_h, &m, areas);
}

stitch_status stitch_lorb(const stitch_image* frame, int32_t m, const int32_t* areas, int32_t fast_threshold,
                          int64_t harris_threshold, int32_t n_max, int32_t nd, const int32_t* pattern,
                          int32_t* counts, int32_t* points, int64_t* responses, uint32_t* descriptors,
                          void* workspace, size_t workspace_bytes, void* stream) {
  if (!frame) return fail(STITCH_E_NULL, "frame is NULL");
  return lorb_run(1, frame, &m, areas, fast_threshold, harris_threshold, n_max, nd, pattern, counts, points,
                  responses, descriptors, workspace, workspace_bytes, stream);
}

stitch_status stitch_lorb_multi(int32_t nframes, const stitch_image* frames, const int32_t* m_per_frame,
                                const int32_t* areas, int32_t fast_threshold, int64_t harris_threshold,
                                int32_t n_max, int32_t nd, const int32_t* pattern, int32_t* counts, int32_t* points,
                                int64_t* responses, uint32_t* descriptors, void* workspace, size_t workspace_bytes,
                                void* stream) {
  if (!frames) return fail(STITCH_E_NULL, "frames is NULL");
  return lorb_run(nframes, frames, m_per_frame, areas, fast_threshold, harris_threshold, n_max, nd, pattern, counts,
                  points, responses, descriptors, workspace, workspace_bytes, stream);
}

}  // extern "C"

namespace {

stitch_status lorb_run(int32_t nframes, const stitch_image* frames, const int32_t* m_per_frame,
                       const int32_t* areas, int32_t fast_threshold, int64_t harris_threshold, int32_t n_max,
                       int32_t nd, const int32_t* pattern, int32_t* counts, int32_t* points, int64_t* responses,
                       uint32_t* descriptors, void* workspace, size_t workspace_bytes, void* stream) {
  if (nframes < 1 || nframes > kMaxFrames) return fail(STITCH_E_SHAPE, "%d frames outside 1..%d", nframes, kMaxFrames);
  int32_t fw[kMaxFrames], fh[kMaxFrames];
  for (int f = 0; f < nframes; ++f) {
    const stitch_status st = check_image(&frames[f], "frame", STITCH_U8, STITCH_HWC, 3);
    if (st) return st;
    fw[f] = frames[f].width;
    fh[f] = frames[f].height;
    if (frames[f].row_pitch * (int64_t)fh[f] >= ((int64_t)1 << 31))
      return fail(STITCH_E_SHAPE, "frame %d spans 2 GiB or more", f);
  }
  if (!pattern || !counts || !points || !responses || !descriptors)
    return fail(STITCH_E_NULL, "pattern or an output is NULL");
  if (nd < 32 || nd > 512 || nd % 32) return fail(STITCH_E_SHAPE, "nd = %d is not a multiple of 32 in 32..512", nd);
  if (n_max < 1 || n_max > (1 << 20)) return fail(STITCH_E_SHAPE, "n_max = %d outside 1..2^20", n_max);
  if (fast_threshold < 0 || fast_threshold > 255) return fail(STITCH_E_SHAPE, "fast_threshold outside 0..255");
  if ((uintptr_t)pattern & 15) return fail(STITCH_E_SHAPE, "pattern is not 16-byte aligned");
  stitch_status st = check_areas(nframes, fw, fh, m_per_frame, areas);
  if (st) return st;
  AreaTable T;
  Layout L;
  if (!plan_areas(nframes, fw, fh, m_per_frame, areas, T, L))
    return fail(STITCH_E_SHAPE, "the areas hold 2^30 samples or more");
  if (!workspace || workspace_bytes < L.bytes || ((uintptr_t)workspace & 255))
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes", L.bytes);
  const int m = T.m;
  T.n_max = n_max;
  T.nd = nd;
  T.pad = 0;
  for (int f = 0; f < kMaxFrames; ++f)
    T.f[f] = f < nframes ? FrameRef{(const uint8_t*)frames[f].data, frames[f].row_pitch, fw[f], fh[f]}
                         : FrameRef{nullptr, 0, 0, 0};
  const hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace;
  int32_t* count = (int32_t*)(ws + L.count);         // per area: survivors, short-list length
  int64_t* listR = (int64_t*)(ws + L.listR);
  int32_t* listI = (int32_t*)(ws + L.listI);
  int64_t* shortR = (int64_t*)(ws + L.shortR);
  int32_t* shortI = (int32_t*)(ws + L.shortI);
  const int tiles = T.a[m - 1].tile_begin + T.a[m - 1].ntiles;
  // optional timing events (taken before anything is enqueued)
  LorbTiming& tm = timing();
  std::array<hipEvent_t, kKinds + 1> ev{};
  bool timed = false;
  {
    std::lock_guard<std::mutex> lock(tm.mu);
    if (tm.on) {
      timed = true;
      for (auto& e : ev) {
        if (!tm.spare.empty()) {
          e = tm.spare.back();
          tm.spare.pop_back();
        } else {
          const hipError_t ce = hipEventCreate(&e);
          if (ce != hipSuccess) return hip_fail(ce, "timing event create");
        }
      }
    }
  }
  hipError_t e = hipSuccess;
  auto mark = [&](int k) {
    if (timed && e == hipSuccess) e = hipEventRecord(ev[k], s);
  };
  mark(0);
  hipLaunchKernelGGL(k_lorb_clear, dim3(1), dim3(128), 0, s, count, m);
  mark(1);
  if (tiles > 0)
    hipLaunchKernelGGL(k_lorb_detect, dim3(tiles), dim3(256), 0, s, T, fast_threshold, harris_threshold, count,
                       listR, listI);
  mark(2);
  hipLaunchKernelGGL(k_lorb_select, dim3(m), dim3(1024), 0, s, T, count, listR, listI, shortR, shortI, counts);
  mark(3);
  hipLaunchKernelGGL(k_lorb_rank, dim3(kRankGrid, m), dim3(256), 0, s, T, count, shortR, shortI, points, responses);
  mark(4);
  hipLaunchKernelGGL(k_lorb_brief, dim3((n_max + 3) / 4, m), dim3(256), 0, s, T, pattern, counts, points,
                     descriptors);
  mark(5);
  if (timed) {
    std::lock_guard<std::mutex> lock(tm.mu);
    if (e == hipSuccess && tm.on) tm.done.push_back(ev);
    else
      for (hipEvent_t x : ev) tm.spare.push_back(x);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "feature extraction launch");
  return STITCH_OK;
}

}  // namespace

extern "C" {

stitch_status stitch_lorb_set_timing(int32_t enable) {
  LorbTiming& tm = timing();
  std::lock_guard<std::mutex> lock(tm.mu);
  tm.on = enable != 0;
  tm.recycle();
  for (int k = 0; k < kKinds; ++k) {
    tm.ms[k] = 0.0;
    tm.n[k] = 0;
  }
  return STITCH_OK;
}

stitch_status stitch_lorb_read_timing(double ms[STITCH_LORB_KINDS], int32_t launches[STITCH_LORB_KINDS]) {
  if (!ms || !launches) return fail(STITCH_E_NULL, "ms or launches is NULL");
  LorbTiming& tm = timing();
  std::lock_guard<std::mutex> lock(tm.mu);
  stitch_status st = STITCH_OK;
  for (auto& c : tm.done) {
    hipError_t e = hipEventSynchronize(c[kKinds]);
    for (int k = 0; e == hipSuccess && k < kKinds; ++k) {
      float t = 0.0f;
      e = hipEventElapsedTime(&t, c[k], c[k + 1]);
      if (e == hipSuccess) {
        tm.ms[k] += t;
        tm.n[k] += 1;
      }
    }
    if (e != hipSuccess && !st) st = hip_fail(e, "timing events");
  }
  tm.recycle();
  for (int k = 0; k < kKinds; ++k) {
    ms[k] = tm.ms[k];
    launches[k] = tm.n[k];
  }
  return st;
}

}  // extern "C"
