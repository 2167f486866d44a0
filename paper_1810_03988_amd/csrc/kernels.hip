// gfx950 kernels of the per-frame stitching path (wave64, LDS-tiled, no MFMA: nothing
// here is a dense contraction; every kernel is bound by HBM traffic).
//
//   k_pyr    fused pyramid pass from level k to k+1 for many cameras at once.  A
//            64x32 level-k tile plus a (4,3)-sample halo is staged in LDS -- at level 0
//            it is produced by the homography warp itself (Alg. 4, step 1), so G_0 never
//            reaches HBM -- then REDUCE gives the level-(k+1) tile with a one-sample halo,
//            EXPAND of that tile is subtracted from G_k to give L_k (multi-band fusion,
//            Sec. 1), and the seam-weight pyramid is reduced in the same pass.
//   k_blend  one level of the synthesis side (Alg. 4, step 6): B_k = sum_i Gm_i L_i and
//            R_k = B_k + EXPAND(R_{k+1}); level 0 writes the uint8 panorama.
//   k_warp, k_warp_coords, k_expand_sub, k_convert: single-stage kernels behind the
//            stitch_warp / stitch_pyramid entry points.
//
// Borders: reflect-101 folded in the fine domain.  Staging the fine tile through the
// periodic reflect-101 extension makes the locally reduced coarse tile equal to the
// fine-domain-folded zero-inserted coarse signal, so EXPAND inside a tile needs no
// border cases at all.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "stitch_internal.h"

namespace stitch {
namespace {

constexpr float kW0 = 1.0f / 16.0f, kW1 = 4.0f / 16.0f, kW2 = 6.0f / 16.0f;
constexpr float kInv255 = 1.0f / 255.0f;

__device__ __forceinline__ float ldv(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const __half* p, int64_t i) { return __half2float(p[i]); }
__device__ __forceinline__ void stv(float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void stv(__half* p, int64_t i, float v) { p[i] = __float2half_rn(v); }

// Periodic reflect-101 extension: index -> [0, n), n >= 2 (period 2(n-1)).
__device__ __forceinline__ int fold(int i, int n) {
  if (i >= 0 && i < n) return i;
  const int p = 2 * (n - 1);
  i %= p;
  if (i < 0) i += p;
  return i < n ? i : p - i;
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a contiguous
// run of logical tiles so neighbouring tiles (which share halos) share an L2.
__device__ __forceinline__ int xcd_remap(int b, int g) {
  const int q = g >> 3, r = g & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// FP32 canvas -> source coordinates: (h0*X + h1*Y) + h2 etc., every operation rounded
// on its own (no contraction into FMA), IEEE divide.
__device__ __forceinline__ void warp_coords(const float* __restrict__ h, int X, int Y, float& x, float& y,
                                            bool& zpos) {
#pragma clang fp contract(off)
  const float Xf = (float)X, Yf = (float)Y;
  const float u = (h[0] * Xf + h[1] * Yf) + h[2];
  const float v = (h[3] * Xf + h[4] * Yf) + h[5];
  const float z = (h[6] * Xf + h[7] * Yf) + h[8];
  zpos = z > 0.0f;
  x = u / z;
  y = v / z;
}

// Bilinear sample of a uint8 HWC RGB frame at the preimage of canvas pixel (X, Y);
// taps outside the frame contribute 0.  Values in [0, 1].
__device__ __forceinline__ void warp_px(const uint8_t* __restrict__ src, int64_t row, int w, int h,
                                        const float* __restrict__ hv, int X, int Y, float out[3]) {
  float x, y;
  bool zpos;
  warp_coords(hv, X, Y, x, y, zpos);
  out[0] = out[1] = out[2] = 0.0f;
  if (!(zpos && x >= -1.0f && x < (float)w && y >= -1.0f && y < (float)h)) return;
  const float x0f = floorf(x), y0f = floorf(y);
  const float fx = x - x0f, fy = y - y0f;
  const int x0 = (int)x0f, y0 = (int)y0f;
  const bool xa = x0 >= 0, xb = x0 + 1 < w, ya = y0 >= 0, yb = y0 + 1 < h;
  const int xc0 = xa ? x0 : 0, xc1 = xb ? x0 + 1 : w - 1;
  const int yc0 = ya ? y0 : 0, yc1 = yb ? y0 + 1 : h - 1;
  const uint8_t* r0 = src + (int64_t)yc0 * row;
  const uint8_t* r1 = src + (int64_t)yc1 * row;
  const float gx = 1.0f - fx, gy = 1.0f - fy;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float p00 = (ya && xa) ? (float)r0[xc0 * 3 + c] : 0.0f;
    const float p01 = (ya && xb) ? (float)r0[xc1 * 3 + c] : 0.0f;
    const float p10 = (yb && xa) ? (float)r1[xc0 * 3 + c] : 0.0f;
    const float p11 = (yb && xb) ? (float)r1[xc1 * 3 + c] : 0.0f;
    out[c] = (gy * (gx * p00 + fx * p01) + fy * (gx * p10 + fx * p11)) * kInv255;
  }
}

__device__ __forceinline__ int find_item(const PyrItem* __restrict__ items, int nitems, int t) {
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------------------------
// Fused pyramid pass.
template <typename T, bool EMIT_LAP>
__global__ void __launch_bounds__(kThreads) k_pyr(const PyrItem* __restrict__ items, int nitems, FrameArgs fa) {
  constexpr int TX = kPyrTX, TY = kPyrTY;
  constexpr int EW = TX + 7, EH = TY + 7;            // fine tile + halo (4 before, 3 after)
  constexpr int CW = TX / 2 + 2, CH = TY / 2 + 2;    // coarse tile + one-sample halo
  __shared__ float sIn[3][EH][EW + 1];
  __shared__ float sH[EH][CW + 1];
  __shared__ float sC[CH][CW + 1];
  __shared__ float sE[CH][TX + 1];

  const int tid = threadIdx.x;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const PyrItem& it = items[find_item(items, nitems, t)];
  const int lt = t - it.tile_begin;
  const int tyi = lt / it.tiles_x, txi = lt - tyi * it.tiles_x;
  const int X0 = it.tile_x0 + txi * TX, Y0 = it.tile_y0 + tyi * TY;   // even
  const int fw = it.fine_w, fh = it.fine_h;
  const int nch = it.nch;

  // ---- stage the fine image tile (all channels) ----
  if (it.img_kind == kSrcWarp) {
    const uint8_t* src = fa.n ? fa.ptr[it.frame_slot] : (const uint8_t*)it.img;
    const int64_t srow = fa.n ? fa.row[it.frame_slot] : it.img_row;
    float hv[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) hv[i] = it.hinv[i];
    for (int e = tid; e < EH * EW; e += kThreads) {
      const int r = e / EW, c = e - r * EW;
      const int Y = fold(Y0 - 4 + r, fh), X = fold(X0 - 4 + c, fw);
      float v[3];
      warp_px(src, srow, it.frame_w, it.frame_h, hv, X, Y, v);
      sIn[0][r][c] = v[0];
      sIn[1][r][c] = v[1];
      sIn[2][r][c] = v[2];
    }
  } else if (it.img_kind == kSrcPlanes) {
    const T* g = (const T*)it.img;
    for (int e = tid; e < EH * EW; e += kThreads) {
      const int r = e / EW, c = e - r * EW;
      const int Y = fold(Y0 - 4 + r, fh) - it.roi_y, X = fold(X0 - 4 + c, fw) - it.roi_x;
      const bool in = X >= 0 && X < it.roi_w && Y >= 0 && Y < it.roi_h;
      const int64_t off = in ? (int64_t)Y * it.img_row + X : 0;
      for (int ch = 0; ch < nch; ++ch) sIn[ch][r][c] = in ? ldv(g, ch * it.img_plane + off) : 0.0f;
    }
  }

  const int cx0 = X0 / 2 - 1, cy0 = Y0 / 2 - 1;    // coarse canvas coords of sC[0][0]
  const bool lap_tile = EMIT_LAP && it.lw_w > 0 && X0 < it.lw_x + it.lw_w && X0 + TX > it.lw_x &&
                        Y0 < it.lw_y + it.lw_h && Y0 + TY > it.lw_y;
  const int nimg = it.img_kind == kSrcNone ? 0 : nch;
  const int npass = nimg + (it.msk_kind != kSrcNone ? 1 : 0);

  for (int ch = 0; ch < npass; ++ch) {
    const bool is_mask = ch >= nimg;
    float(*in)[EW + 1] = sIn[is_mask ? 0 : ch];
    if (is_mask) {
      __syncthreads();   // sIn[0] may still be read by the previous channel's subtract
      if (it.msk_kind == kSrcU8) {
        const uint8_t* m = (const uint8_t*)it.msk;
        for (int e = tid; e < EH * EW; e += kThreads) {
          const int r = e / EW, c = e - r * EW;
          const int Y = fold(Y0 - 4 + r, fh) - it.roi_y, X = fold(X0 - 4 + c, fw) - it.roi_x;
          const bool inr = X >= 0 && X < it.roi_w && Y >= 0 && Y < it.roi_h;
          in[r][c] = inr ? (float)m[(int64_t)Y * it.msk_row + X] * kInv255 : 0.0f;
        }
      } else {
        const T* m = (const T*)it.msk;
        for (int e = tid; e < EH * EW; e += kThreads) {
          const int r = e / EW, c = e - r * EW;
          const int Y = fold(Y0 - 4 + r, fh) - it.roi_y, X = fold(X0 - 4 + c, fw) - it.roi_x;
          const bool inr = X >= 0 && X < it.roi_w && Y >= 0 && Y < it.roi_h;
          in[r][c] = inr ? ldv(m, (int64_t)Y * it.msk_row + X) : 0.0f;
        }
      }
    }
    __syncthreads();
    // ---- REDUCE, horizontal: every staged row, coarse columns cx0 .. cx0+CW-1 ----
    for (int e = tid; e < EH * CW; e += kThreads) {
      const int r = e / CW, j = e - r * CW;
      const float* s = &in[r][2 * j];
      sH[r][j] = kW0 * (s[0] + s[4]) + kW1 * (s[1] + s[3]) + kW2 * s[2];
    }
    __syncthreads();
    // ---- REDUCE, vertical -> extended coarse tile; store its interior ----
    T* gout = (T*)(is_mask ? it.gm_out : it.g_out);
    const int64_t grow = is_mask ? it.gm_row : it.g_row;
    const int64_t gplane = is_mask ? 0 : (int64_t)ch * it.g_plane;
    for (int e = tid; e < CH * CW; e += kThreads) {
      const int i = e / CW, j = e - i * CW;
      const float* s = &sH[2 * i][j];
      constexpr int S = CW + 1;
      const float v = kW0 * (s[0] + s[4 * S]) + kW1 * (s[S] + s[3 * S]) + kW2 * s[2 * S];
      sC[i][j] = v;
      const int cy = cy0 + i - it.croi_y, cx = cx0 + j - it.croi_x;
      if (i >= 1 && i <= TY / 2 && j >= 1 && j <= TX / 2 && cy >= 0 && cy < it.croi_h && cx >= 0 &&
          cx < it.croi_w && gout != nullptr)
        stv(gout, gplane + (int64_t)cy * grow + cx, v);
    }
    if (is_mask || !lap_tile) continue;
    __syncthreads();
    // ---- EXPAND, horizontal: coarse rows x fine columns (interior form) ----
    for (int e = tid; e < CH * TX; e += kThreads) {
      const int i = e / TX, x = e - i * TX;
      const float* s = &sC[i][x >> 1];
      sE[i][x] = (x & 1) ? 0.5f * (s[1] + s[2]) : 0.125f * (s[0] + s[2]) + 0.75f * s[1];
    }
    __syncthreads();
    // ---- EXPAND, vertical, and L_k = G_k - EXPAND(G_{k+1}) on the band window ----
    T* lout = (T*)it.l_out;
    for (int e = tid; e < TY * TX; e += kThreads) {
      const int y = e / TX, x = e - y * TX;
      const float* s = &sE[y >> 1][x];
      constexpr int S = TX + 1;
      const float ev = (y & 1) ? 0.5f * (s[S] + s[2 * S]) : 0.125f * (s[0] + s[2 * S]) + 0.75f * s[S];
      const int Y = Y0 + y - it.lw_y, X = X0 + x - it.lw_x;
      if (X >= 0 && X < it.lw_w && Y >= 0 && Y < it.lw_h)
        stv(lout, (int64_t)ch * it.l_plane + (int64_t)Y * it.l_row + X, in[y + 4][x + 4] - ev);
    }
  }
}

// ------------------------------------------------------------------------------------
// One synthesis level: B_k over cameras + EXPAND(R_{k+1}) -> R_k (and the panorama at k = 0).
template <typename T, bool FINAL, bool HAS_COARSE>
__global__ void __launch_bounds__(kThreads) k_blend(BlendArgs a) {
  constexpr int TX = kBlendTX, TY = kBlendTY;
  constexpr int CW = TX / 2 + 2, CH = TY / 2 + 2;
  __shared__ float sC[3][CH][CW + 1];
  __shared__ float sE[3][CH][TX + 1];
  __shared__ int sCam[kMaxCameras];
  __shared__ int sNCam;

  const int tid = threadIdx.x;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int tyi = t / a.tiles_x, txi = t - tyi * a.tiles_x;
  const int X0 = txi * TX, Y0 = tyi * TY;

  if (tid == 0) {
    int m = 0;
    for (int i = 0; i < a.ncam; ++i) {
      const BlendCam& c = a.cams[i];
      const int x0 = max(c.lx, c.wx), x1 = min(c.lx + c.lw, c.wx + c.ww);
      const int y0 = max(c.ly, c.wy), y1 = min(c.ly + c.lh, c.wy + c.wh);
      if (x0 < x1 && y0 < y1 && x0 < X0 + TX && x1 > X0 && y0 < Y0 + TY && y1 > Y0) sCam[m++] = i;
    }
    sNCam = m;
  }
  if (HAS_COARSE) {
    const T* r = (const T*)a.r_in;
    const int cx0 = X0 / 2 - 1, cy0 = Y0 / 2 - 1;
    for (int e = tid; e < CH * CW; e += kThreads) {
      const int i = e / CW, j = e - i * CW;
      // coarse index of the fine-domain fold of fine sample 2*c, kept inside the level
      const int cy = min(fold(2 * (cy0 + i), a.H) >> 1, a.cH - 1);
      const int cx = min(fold(2 * (cx0 + j), a.W) >> 1, a.cW - 1);
      const int64_t off = (int64_t)cy * a.rin_row + cx;
#pragma unroll
      for (int c = 0; c < 3; ++c) sC[c][i][j] = ldv(r, c * a.rin_plane + off);
    }
    __syncthreads();
    for (int e = tid; e < 3 * CH * TX; e += kThreads) {
      const int c = e / (CH * TX), rem = e - c * CH * TX;
      const int i = rem / TX, x = rem - i * TX;
      const float* s = &sC[c][i][x >> 1];
      sE[c][i][x] = (x & 1) ? 0.5f * (s[1] + s[2]) : 0.125f * (s[0] + s[2]) + 0.75f * s[1];
    }
  }
  __syncthreads();
  const int ncam = sNCam;
  for (int e = tid; e < TY * TX; e += kThreads) {
    const int y = e / TX, x = e - y * TX;
    const int X = X0 + x, Y = Y0 + y;
    if (X >= a.W || Y >= a.H) continue;
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (int q = 0; q < ncam; ++q) {
      const BlendCam& c = a.cams[sCam[q]];
      const int lx = X - c.lx, ly = Y - c.ly, wx = X - c.wx, wy = Y - c.wy;
      if (lx < 0 || lx >= c.lw || ly < 0 || ly >= c.lh || wx < 0 || wx >= c.ww || wy < 0 || wy >= c.wh) continue;
      const float wgt = c.wgt_u8 ? (float)((const uint8_t*)c.wgt)[(int64_t)wy * c.wgt_row + wx] * kInv255
                                 : ldv((const T*)c.wgt, (int64_t)wy * c.wgt_row + wx);
      const T* l = (const T*)c.lap;
      const int64_t off = (int64_t)ly * c.lap_row + lx;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) acc[ch] = acc[ch] + wgt * ldv(l, ch * c.lap_plane + off);
    }
    if (HAS_COARSE) {
      constexpr int S = TX + 1;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float* s = &sE[ch][y >> 1][x];
        const float ev = (y & 1) ? 0.5f * (s[S] + s[2 * S]) : 0.125f * (s[0] + s[2 * S]) + 0.75f * s[S];
        acc[ch] = acc[ch] + ev;
      }
    }
    if (a.r_out != nullptr) {
      T* ro = (T*)a.r_out;
      const int64_t off = (int64_t)Y * a.rout_row + X;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) stv(ro, ch * a.rout_plane + off, acc[ch]);
    }
    if (FINAL) {
      uint8_t* p = a.pano + (int64_t)Y * a.pano_row + (int64_t)X * 3;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) p[ch] = (uint8_t)fminf(fmaxf(rintf(255.0f * acc[ch]), 0.0f), 255.0f);
    }
  }
}

// ------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) k_warp(const uint8_t* __restrict__ src, int64_t srow, int w, int h,
                                                   Hinv9 hi, int rx, int ry, T* __restrict__ dst, int64_t drow,
                                                   int64_t dplane, int dw, int dh) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= dw || y >= dh) return;
  float v[3];
  warp_px(src, srow, w, h, hi.h, rx + x, ry + y, v);
  const int64_t off = (int64_t)y * drow + x;
#pragma unroll
  for (int c = 0; c < 3; ++c) stv(dst, c * dplane + off, v[c]);
}

__global__ void __launch_bounds__(kThreads) k_warp_coords(Hinv9 hi, int rx, int ry, float* __restrict__ dst,
                                                          int64_t drow, int64_t dplane, int dw, int dh) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= dw || y >= dh) return;
  float sx, sy;
  bool zpos;
  warp_coords(hi.h, rx + x, ry + y, sx, sy, zpos);
  const int64_t off = (int64_t)y * drow + x;
  dst[off] = zpos ? sx : __builtin_nanf("");
  dst[dplane + off] = zpos ? sy : __builtin_nanf("");
}

// In place: fine <- fine - EXPAND(coarse) on the fine rectangle; both levels are zero
// outside their rectangles; fine-domain reflect-101 on the level-k canvas (cw x ch).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_expand_sub(int nch, T* __restrict__ f, int64_t frow, int64_t fplane,
                                                         int fx0, int fy0, int fwid, int fhei,
                                                         const T* __restrict__ g, int64_t grow, int64_t gplane,
                                                         int gx0, int gy0, int gwid, int ghei, int W, int H) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= fwid || y >= fhei) return;
  const int X = fx0 + x, Y = fy0 + y;
  const float w2[5] = {2.0f * kW0, 2.0f * kW1, 2.0f * kW2, 2.0f * kW1, 2.0f * kW0};
  for (int c = 0; c < nch; ++c) {
    float e = 0.0f;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const int ty = fold(Y + a - 2, H);
      if (ty & 1) continue;
      const int cy = (ty >> 1) - gy0;
      if (cy < 0 || cy >= ghei) continue;
      float row = 0.0f;
#pragma unroll
      for (int b = 0; b < 5; ++b) {
        const int tx = fold(X + b - 2, W);
        if (tx & 1) continue;
        const int cx = (tx >> 1) - gx0;
        if (cx < 0 || cx >= gwid) continue;
        row += w2[b] * ldv(g, c * gplane + (int64_t)cy * grow + cx);
      }
      e += w2[a] * row;
    }
    const int64_t off = c * fplane + (int64_t)y * frow + x;
    stv(f, off, ldv(f, off) - e);
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_convert(int nch, int src_u8, const void* __restrict__ s, int64_t srow,
                                                      int64_t splane, T* __restrict__ d, int64_t drow,
                                                      int64_t dplane, int w, int h) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= w || y >= h) return;
  for (int c = 0; c < nch; ++c) {
    const float v = src_u8 ? (float)((const uint8_t*)s)[c * splane + (int64_t)y * srow + x] * kInv255
                           : ldv((const T*)s, c * splane + (int64_t)y * srow + x);
    stv(d, c * dplane + (int64_t)y * drow + x, v);
  }
}

}  // namespace

// ------------------------------------------------------------------------------------ launchers
hipError_t launch_pyr(bool f16, bool emit_lap, const PyrItem* items_dev, int nitems, int total_tiles,
                      const FrameArgs& fa, hipStream_t s) {
  if (total_tiles <= 0) return hipSuccess;
  const dim3 grid(total_tiles), block(kThreads);
  if (f16) {
    if (emit_lap) hipLaunchKernelGGL((k_pyr<__half, true>), grid, block, 0, s, items_dev, nitems, fa);
    else hipLaunchKernelGGL((k_pyr<__half, false>), grid, block, 0, s, items_dev, nitems, fa);
  } else {
    if (emit_lap) hipLaunchKernelGGL((k_pyr<float, true>), grid, block, 0, s, items_dev, nitems, fa);
    else hipLaunchKernelGGL((k_pyr<float, false>), grid, block, 0, s, items_dev, nitems, fa);
  }
  return hipGetLastError();
}

hipError_t launch_blend(bool f16, const BlendArgs& a, hipStream_t s) {
  const int tiles = a.tiles_x * a.tiles_y;
  if (tiles <= 0) return hipSuccess;
  const dim3 grid(tiles), block(kThreads);
  const bool fin = a.pano != nullptr;
  const bool co = a.has_coarse != 0;
#define STITCH_BLEND(TT)                                                                        \
  do {                                                                                          \
    if (fin && co) hipLaunchKernelGGL((k_blend<TT, true, true>), grid, block, 0, s, a);         \
    else if (fin) hipLaunchKernelGGL((k_blend<TT, true, false>), grid, block, 0, s, a);         \
    else if (co) hipLaunchKernelGGL((k_blend<TT, false, true>), grid, block, 0, s, a);          \
    else hipLaunchKernelGGL((k_blend<TT, false, false>), grid, block, 0, s, a);                 \
  } while (0)
  if (f16) STITCH_BLEND(__half);
  else STITCH_BLEND(float);
#undef STITCH_BLEND
  return hipGetLastError();
}

hipError_t launch_warp(bool f16, const uint8_t* src, int64_t src_row, int w, int h, const float* hinv9, int roi_x,
                       int roi_y, void* dst, int64_t dst_row, int64_t dst_plane, int dw, int dh, hipStream_t s) {
  if (dw <= 0 || dh <= 0) return hipSuccess;
  Hinv9 hi;
  for (int i = 0; i < 9; ++i) hi.h[i] = hinv9[i];
  const dim3 grid((dw + 63) / 64, (dh + 3) / 4), block(kThreads);
  if (f16)
    hipLaunchKernelGGL((k_warp<__half>), grid, block, 0, s, src, src_row, w, h, hi, roi_x, roi_y, (__half*)dst,
                       dst_row, dst_plane, dw, dh);
  else
    hipLaunchKernelGGL((k_warp<float>), grid, block, 0, s, src, src_row, w, h, hi, roi_x, roi_y, (float*)dst,
                       dst_row, dst_plane, dw, dh);
  return hipGetLastError();
}

hipError_t launch_warp_coords(const float* hinv9, int roi_x, int roi_y, float* dst, int64_t row, int64_t plane,
                              int dw, int dh, hipStream_t s) {
  if (dw <= 0 || dh <= 0) return hipSuccess;
  Hinv9 hi;
  for (int i = 0; i < 9; ++i) hi.h[i] = hinv9[i];
  const dim3 grid((dw + 63) / 64, (dh + 3) / 4), block(kThreads);
  hipLaunchKernelGGL(k_warp_coords, grid, block, 0, s, hi, roi_x, roi_y, dst, row, plane, dw, dh);
  return hipGetLastError();
}

hipError_t launch_expand_sub(bool f16, int nch, void* fine, int64_t f_row, int64_t f_plane, int fx, int fy, int fw,
                             int fh, const void* coarse, int64_t c_row, int64_t c_plane, int cx, int cy, int cw,
                             int ch, int canvas_w, int canvas_h, hipStream_t s) {
  if (fw <= 0 || fh <= 0) return hipSuccess;
  const dim3 grid((fw + 63) / 64, (fh + 3) / 4), block(kThreads);
  if (f16)
    hipLaunchKernelGGL((k_expand_sub<__half>), grid, block, 0, s, nch, (__half*)fine, f_row, f_plane, fx, fy, fw,
                       fh, (const __half*)coarse, c_row, c_plane, cx, cy, cw, ch, canvas_w, canvas_h);
  else
    hipLaunchKernelGGL((k_expand_sub<float>), grid, block, 0, s, nch, (float*)fine, f_row, f_plane, fx, fy, fw, fh,
                       (const float*)coarse, c_row, c_plane, cx, cy, cw, ch, canvas_w, canvas_h);
  return hipGetLastError();
}

hipError_t launch_convert(bool f16_out, int nch, bool src_u8, const void* src, int64_t s_row, int64_t s_plane,
                          void* dst, int64_t d_row, int64_t d_plane, int w, int h, hipStream_t s) {
  if (w <= 0 || h <= 0) return hipSuccess;
  const dim3 grid((w + 63) / 64, (h + 3) / 4), block(kThreads);
  if (f16_out)
    hipLaunchKernelGGL((k_convert<__half>), grid, block, 0, s, nch, (int)src_u8, src, s_row, s_plane,
                       (__half*)dst, d_row, d_plane, w, h);
  else
    hipLaunchKernelGGL((k_convert<float>), grid, block, 0, s, nch, (int)src_u8, src, s_row, s_plane,
                       (float*)dst, d_row, d_plane, w, h);
  return hipGetLastError();
}

}  // namespace stitch
