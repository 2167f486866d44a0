// L-ORB feature extraction on gfx950 (Sec. 4.1, Alg. 1 and Alg. 2): in each feature
// detection area of a frame, FAST corners scored by the Harris response, non-maximal
// suppression, the N strongest, and their BRIEF descriptors.  All decisions are exact
// integer arithmetic:
//   gray level      g = (77 R + 150 G + 29 B + 128) >> 8
//   FAST            >= 9 contiguous pixels of the radius-3 circle brighter than g + tf or
//                   darker than g - tf
//   Harris          central-difference gradients, 5x5 binomial window b b^T (sigma = 1),
//                   R = 64 (A B - C^2) - 3 (A + B)^2  (alpha = 3/64, scaled by 64), int64
//   candidates      FAST corners with R > t; suppression over 3x3 among candidates, ties
//                   to the first in raster order; the N of largest R, ties by raster order
//   BRIEF           three-valued tests of n_d point pairs on S = b b^T * g (integer sums),
//                   kept as a "greater" and a "less" bit string
// Points must keep their descriptor support in the frame (17 samples from every edge);
// areas are clipped to that range.
//
// Per area: k_lorb_response (64x16 tiles, the gray tile and its 3-sample halo in LDS,
// gradient products and the separable window in LDS) -> k_lorb_suppress (sort keys:
// R with its sign bit flipped for survivors, 0 otherwise, and a survivor count) -> a
// stable descending radix sort (hipCUB), which keeps raster order among equal keys ->
// k_lorb_brief (one wave per kept point).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>

#include "stitch_internal.h"

using namespace stitch;

namespace {

constexpr int kMargin = 17;
constexpr int kLTX = 64, kLTY = 16, kHalo = 3;
constexpr int kGW = kLTX + 2 * kHalo, kGH = kLTY + 2 * kHalo;      // 70 x 22 gray tile
constexpr int kDW = kLTX + 4, kDH = kLTY + 4;                       // 68 x 20 gradient products
constexpr int64_t kNone = INT64_MIN;
constexpr uint64_t kSign = 0x8000000000000000ull;

__device__ __forceinline__ int luma(const uint8_t* p) {
  return (77 * (int)p[0] + 150 * (int)p[1] + 29 * (int)p[2] + 128) >> 8;
}

// FAST circle of radius 3, clockwise from the top
__constant__ int8_t kCircle[16][2] = {{0, -3}, {1, -3}, {2, -2}, {3, -1}, {3, 0}, {3, 1}, {2, 2}, {1, 3},
                                      {0, 3}, {-1, 3}, {-2, 2}, {-3, 1}, {-3, 0}, {-3, -1}, {-2, -2}, {-1, -3}};

struct Area {
  int x0, y0, w, h;       // clipped area (frame coordinates)
};

__global__ void __launch_bounds__(256) k_lorb_response(const uint8_t* __restrict__ frame, int64_t row, int fw, int fh,
                                                       Area a, int tf, int64_t t, int64_t* __restrict__ R,
                                                       int32_t* __restrict__ count) {
  __shared__ int sG[kGH][kGW + 2];
  __shared__ int sP[3][kDH][kDW];          // Ix^2, Iy^2, Ix Iy
  __shared__ int sH[3][kDH][kLTX];         // horizontally weighted
  const int tid = threadIdx.x;
  const int ox = blockIdx.x * kLTX, oy = blockIdx.y * kLTY;   // tile origin in the area
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) *count = 0;   // survivors of this area
  // gray tile with a 3-sample halo (coordinates clamped into the frame: samples past the
  // area's far edges only feed outputs that are not written)
  for (int e = tid; e < kGH * kGW; e += 256) {
    const int r = e / kGW, c = e - r * kGW;
    const int x = min(a.x0 + ox - kHalo + c, fw - 1), y = min(a.y0 + oy - kHalo + r, fh - 1);
    sG[r][c] = luma(frame + (int64_t)y * row + 3 * (int64_t)x);
  }
  __syncthreads();
  // central-difference gradients and their products on the 68 x 20 inner window
  for (int e = tid; e < kDH * kDW; e += 256) {
    const int r = e / kDW, c = e - r * kDW;
    const int gr = r + 1, gc = c + 1;
    const int ix = sG[gr][gc + 1] - sG[gr][gc - 1], iy = sG[gr + 1][gc] - sG[gr - 1][gc];
    sP[0][r][c] = ix * ix;
    sP[1][r][c] = iy * iy;
    sP[2][r][c] = ix * iy;
  }
  __syncthreads();
  // binomial window [1 4 6 4 1], horizontally
  for (int e = tid; e < 3 * kDH * kLTX; e += 256) {
    const int q = e / (kDH * kLTX), rem = e - q * (kDH * kLTX);
    const int r = rem / kLTX, c = rem - r * kLTX;
    const int* p = &sP[q][r][c];
    sH[q][r][c] = (p[0] + p[4]) + 4 * (p[1] + p[3]) + 6 * p[2];
  }
  __syncthreads();
  // vertically, the response and the FAST test: four outputs per thread
  for (int e = tid; e < kLTX * kLTY; e += 256) {
    const int r = e / kLTX, c = e - r * kLTX;
    const int x = ox + c, y = oy + r;
    if (x >= a.w || y >= a.h) continue;
    int64_t m[3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
      m[q] = (int64_t)(sH[q][r][c] + sH[q][r + 4][c]) + 4 * (int64_t)(sH[q][r + 1][c] + sH[q][r + 3][c]) +
             6 * (int64_t)sH[q][r + 2][c];
    const int64_t A = m[0], B = m[1], C = m[2];
    const int64_t resp = 64 * (A * B - C * C) - 3 * (A + B) * (A + B);
    const int gr = r + kHalo, gc = c + kHalo;
    const int p = sG[gr][gc];
    unsigned bright = 0, dark = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int v = sG[gr + kCircle[k][1]][gc + kCircle[k][0]];
      bright |= (unsigned)(v > p + tf) << k;
      dark |= (unsigned)(v < p - tf) << k;
    }
    // 9 contiguous set bits somewhere on the (cyclic) circle
    auto run9 = [](unsigned m16) {
      unsigned m = m16 | (m16 << 16);
#pragma unroll
      for (int s = 1; s < 9; ++s) m &= m >> 1;   // bit i set: bits i .. i+8 all set
      return (m & 0xFFFFu) != 0;
    };
    const bool cand = (run9(bright) || run9(dark)) && resp > t;
    R[(int64_t)y * a.w + x] = cand ? resp : kNone;
  }
}

__global__ void __launch_bounds__(256) k_lorb_suppress(const int64_t* __restrict__ R, Area a,
                                                       uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                                                       int32_t* __restrict__ count) {
  const int64_t n = (int64_t)a.w * a.h;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / a.w), x = (int)(i - (int64_t)y * a.w);
  const int64_t r = R[i];
  bool keep = r != kNone;
  if (keep) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (!dx && !dy) continue;
        const int qx = x + dx, qy = y + dy;
        if (qx < 0 || qx >= a.w || qy < 0 || qy >= a.h) continue;
        const int64_t j = (int64_t)qy * a.w + qx;
        const int64_t rq = R[j];
        if (rq != kNone && !(rq < r || (rq == r && j > i))) keep = false;
      }
  }
  keys[i] = keep ? ((uint64_t)r ^ kSign) : 0ull;
  vals[i] = (int32_t)i;
  if (keep) atomicAdd(count, 1);
}

// One wave per kept point k (k < min(count, n_max)): 64 lanes evaluate the pattern's pairs
// lane, lane + 64, ...; S at a point is the 5x5 binomial sum of the gray levels.  Pattern
// offsets are clamped to +-15 so that every read stays in the frame.  empty: the area
// holds no sample (count was not written).
__global__ void __launch_bounds__(64) k_lorb_brief(const uint8_t* __restrict__ frame, int64_t row, Area a,
                                                   const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals,
                                                   const int32_t* __restrict__ count, int empty, int n_max, int nd,
                                                   const int32_t* __restrict__ pattern, int32_t* __restrict__ counts_out,
                                                   int32_t* __restrict__ pts, int64_t* __restrict__ resp,
                                                   uint32_t* __restrict__ desc) {
  const int k = blockIdx.x, lane = threadIdx.x;
  const int nk = empty ? 0 : min(*count, n_max);
  if (k == 0 && lane == 0) *counts_out = nk;
  if (k >= nk) return;
  const int idx = vals[k];
  const int y = a.y0 + idx / a.w, x = a.x0 + idx % a.w;
  if (lane == 0) {
    pts[2 * k] = x;
    pts[2 * k + 1] = y;
    resp[k] = (int64_t)(keys[k] ^ kSign);
  }
  auto S = [&](int px, int py) {
    const int b[5] = {1, 4, 6, 4, 1};
    int s = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const uint8_t* rp = frame + (int64_t)(py + j - 2) * row + 3 * (int64_t)(px - 2);
      int h = 0;
#pragma unroll
      for (int i = 0; i < 5; ++i) h += b[i] * luma(rp + 3 * i);
      s += b[j] * h;
    }
    return s;
  };
  const int words = nd / 32;
  for (int base = 0; base < nd; base += 64) {
    const int pk = base + lane;
    bool gt = false, lt = false;
    if (pk < nd) {
      const int32_t* pp = pattern + 4 * pk;
      auto off = [](int32_t v) { return min(max(v, -15), 15); };
      const int s1 = S(x + off(pp[0]), y + off(pp[1])), s2 = S(x + off(pp[2]), y + off(pp[3]));
      gt = s1 > s2;
      lt = s1 < s2;
    }
    const uint64_t mg = __ballot(gt), ml = __ballot(lt);
    if (lane == 0) {
      uint32_t* d = desc + (int64_t)k * 2 * words;
      const int w0 = base / 32;
      d[w0] = (uint32_t)mg;
      d[words + w0] = (uint32_t)ml;
      if (w0 + 1 < words) {
        d[w0 + 1] = (uint32_t)(mg >> 32);
        d[words + w0 + 1] = (uint32_t)(ml >> 32);
      }
    }
  }
}

Area clip(const int32_t* r, int fw, int fh) {
  Area a;
  const int x1 = std::min(r[0] + r[2], fw - kMargin), y1 = std::min(r[1] + r[3], fh - kMargin);
  a.x0 = std::max(r[0], kMargin);
  a.y0 = std::max(r[1], kMargin);
  a.w = std::max(0, x1 - a.x0);
  a.h = std::max(0, y1 - a.y0);
  return a;
}

int64_t largest_area(int fw, int fh, int32_t m, const int32_t* areas) {
  int64_t n = 0;
  for (int i = 0; i < m; ++i) {
    const Area a = clip(areas + 4 * i, fw, fh);
    n = std::max(n, (int64_t)a.w * a.h);
  }
  return n;
}

size_t up(size_t v) { return (v + 255) & ~(size_t)255; }

// workspace layout for areas of at most n samples
struct LorbLayout {
  size_t r, keys_in, keys_out, vals_in, vals_out, count, temp, temp_bytes, total;
};

bool layout(int64_t n, LorbLayout& L) {
  size_t tb = 0;
  if (hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tb, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                                   (int32_t*)nullptr, (int32_t*)nullptr, (int)std::max<int64_t>(n, 1),
                                                   0, 64) != hipSuccess)
    return false;
  size_t o = 0;
  L.r = o; o += up((size_t)n * 8);
  L.keys_in = o; o += up((size_t)n * 8);
  L.keys_out = o; o += up((size_t)n * 8);
  L.vals_in = o; o += up((size_t)n * 4);
  L.vals_out = o; o += up((size_t)n * 4);
  L.count = o; o += 256;
  L.temp = o; o += up(tb);
  L.temp_bytes = tb;
  L.total = o;
  return true;
}

}  // namespace

extern "C" {

size_t stitch_lorb_workspace_bytes(int32_t frame_w, int32_t frame_h, int32_t m, const int32_t* areas) {
  if (m < 1 || !areas || frame_w < 1 || frame_h < 1) return 0;
  LorbLayout L;
  if (!layout(std::max<int64_t>(largest_area(frame_w, frame_h, m, areas), 1), L)) {
    fail(STITCH_E_DEVICE, "the sort's storage query failed (no usable device?)");
    return 0;
  }
  return L.total;
}

stitch_status stitch_lorb(const stitch_image* frame, int32_t m, const int32_t* areas, int32_t fast_threshold,
                          int64_t harris_threshold, int32_t n_max, int32_t nd, const int32_t* pattern,
                          int32_t* counts, int32_t* points, int64_t* responses, uint32_t* descriptors,
                          void* workspace, size_t workspace_bytes, void* stream) {
  stitch_status st = check_image(frame, "frame", STITCH_U8, STITCH_HWC, 3);
  if (st) return st;
  if (m < 1 || m > 64) return fail(STITCH_E_SHAPE, "m = %d areas outside 1..64", m);
  if (!areas || !pattern || !counts || !points || !responses || !descriptors)
    return fail(STITCH_E_NULL, "areas, pattern or an output is NULL");
  if (nd < 32 || nd > 512 || nd % 32) return fail(STITCH_E_SHAPE, "nd = %d is not a multiple of 32 in 32..512", nd);
  if (n_max < 1 || n_max > (1 << 20)) return fail(STITCH_E_SHAPE, "n_max = %d outside 1..2^20", n_max);
  if (fast_threshold < 0 || fast_threshold > 255) return fail(STITCH_E_SHAPE, "fast_threshold outside 0..255");
  const int fw = frame->width, fh = frame->height;
  if (fw < 2 * kMargin + 1 || fh < 2 * kMargin + 1)
    return fail(STITCH_E_SHAPE, "frames need at least %d samples per side", 2 * kMargin + 1);
  if (frame->row_pitch * (int64_t)fh >= ((int64_t)1 << 31))
    return fail(STITCH_E_SHAPE, "frame spans 2 GiB or more");
  for (int i = 0; i < m; ++i)
    if (areas[4 * i + 2] < 0 || areas[4 * i + 3] < 0) return fail(STITCH_E_SHAPE, "area %d has a negative size", i);
  const int64_t nmax_area = largest_area(fw, fh, m, areas);
  if (nmax_area >= ((int64_t)1 << 30)) return fail(STITCH_E_SHAPE, "an area holds 2^30 samples or more");
  LorbLayout L;
  if (!layout(std::max<int64_t>(nmax_area, 1), L)) return fail(STITCH_E_DEVICE, "sort storage query failed");
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace & 255))
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes", L.total);
  const hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace;
  const uint8_t* src = (const uint8_t*)frame->data;
  const int words = nd / 32;
  for (int i = 0; i < m; ++i) {
    const Area a = clip(areas + 4 * i, fw, fh);
    int32_t* cnt_out = counts + i;
    int32_t* pts = points + (int64_t)i * n_max * 2;
    int64_t* rsp = responses + (int64_t)i * n_max;
    uint32_t* dsc = descriptors + (int64_t)i * n_max * 2 * words;
    int32_t* count = (int32_t*)(ws + L.count);
    hipError_t e = hipSuccess;
    const int64_t n = (int64_t)a.w * a.h;
    if (n > 0) {
      int64_t* R = (int64_t*)(ws + L.r);
      hipLaunchKernelGGL(k_lorb_response, dim3((a.w + kLTX - 1) / kLTX, (a.h + kLTY - 1) / kLTY), dim3(256), 0, s, src,
                         frame->row_pitch, fw, fh, a, fast_threshold, harris_threshold, R, count);
      e = hipGetLastError();
      uint64_t* kin = (uint64_t*)(ws + L.keys_in);
      int32_t* vin = (int32_t*)(ws + L.vals_in);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_lorb_suppress, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, R, a, kin, vin, count);
        e = hipGetLastError();
      }
      if (e == hipSuccess) {
        size_t tb = L.temp_bytes;
        e = hipcub::DeviceRadixSort::SortPairsDescending(ws + L.temp, tb, kin, (uint64_t*)(ws + L.keys_out), vin,
                                                         (int32_t*)(ws + L.vals_out), (int)n, 0, 64, s);
      }
    }
    if (e == hipSuccess) {
      // n == 0: one block only records the zero count
      hipLaunchKernelGGL(k_lorb_brief, dim3(n > 0 ? n_max : 1), dim3(64), 0, s, src, frame->row_pitch, a,
                         (const uint64_t*)(ws + L.keys_out), (const int32_t*)(ws + L.vals_out), count, n == 0, n_max, nd,
                         pattern, cnt_out, pts, rsp, dsc);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_fail(e, "feature extraction launch");
  }
  return STITCH_OK;
}

}  // extern "C"
