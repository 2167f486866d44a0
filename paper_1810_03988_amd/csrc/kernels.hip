// gfx950 kernels of the per-frame stitching path (wave64, LDS-tiled, no MFMA: nothing
// here is a dense contraction; every kernel is bound by HBM traffic).
//
//   k_pyr    fused pyramid pass from level k to k+1 for many cameras at once.  A
//            64-column level-k tile is walked in 16-row sub-steps; each is staged in LDS
//            with a (4,3)-sample halo -- at level 0 it is produced by the homography warp
//            itself (Alg. 4, step 1), so G_0 never reaches HBM -- then REDUCE gives the
//            level-(k+1) tile with a one-sample halo,
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
#include <hip/hip_runtime.h>

#include <cstring>

#include "stitch_internal.h"

namespace stitch {
namespace {

constexpr float kW0 = 1.0f / 16.0f, kW1 = 4.0f / 16.0f, kW2 = 6.0f / 16.0f;
constexpr float kInv255 = 1.0f / 255.0f;

#define GLB __attribute__((address_space(1)))
#define CST __attribute__((address_space(4)))

// Descriptor tables are written by the host before a launch and never during it: read them
// through the constant address space, so uniform reads become scalar loads.
template <typename T>
__device__ __forceinline__ const CST T* cst(const T* p) { return (const CST T*)p; }
// A whole descriptor by value (dword copies, merged into wide scalar loads).
template <typename T>
__device__ __forceinline__ T ld_cst(const CST T* p) {
  static_assert(sizeof(T) % 4 == 0, "descriptors are dword multiples");
  T v;
  uint32_t* d = reinterpret_cast<uint32_t*>(&v);
  const CST uint32_t* s = reinterpret_cast<const CST uint32_t*>(p);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = s[i];
  return v;
}

// Views of descriptor-held pointers as global memory, so accesses compile to global (not
// flat) instructions.
template <typename T>
__device__ __forceinline__ const GLB T* cg(const void* p) { return (const GLB T*)p; }
template <typename T>
__device__ __forceinline__ GLB T* mg(void* p) { return (GLB T*)p; }
__device__ __forceinline__ float ldg(const GLB float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldg(const GLB _Float16* p, int64_t i) { return (float)p[i]; }
__device__ __forceinline__ void stg(GLB float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void stg(GLB _Float16* p, int64_t i, float v) { p[i] = (_Float16)v; }

// Raw bits of a stored sample (zero-extended), converted separately: loads can then all be
// issued before the first conversion.
template <typename T> struct RawOf;
template <> struct RawOf<float> { using type = uint32_t; };
template <> struct RawOf<_Float16> { using type = uint16_t; };
template <typename T>
__device__ __forceinline__ typename RawOf<T>::type ld_raw(const GLB T* p, int64_t i) {
  return *(const GLB typename RawOf<T>::type*)(p + i);
}
__device__ __forceinline__ float from_raw(uint32_t b) { return __builtin_bit_cast(float, b); }
__device__ __forceinline__ float from_raw(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef _Float16 vh4 __attribute__((ext_vector_type(4)));

// Streaming stores for the pyramid levels (written once, read by a later kernel long after
// the lines would have left L2); the four-sample forms need 4-sample alignment (checked by
// the caller).
__device__ __forceinline__ void stgnt(GLB float* p, int64_t i, float v) { __builtin_nontemporal_store(v, p + i); }
__device__ __forceinline__ void stgnt(GLB _Float16* p, int64_t i, float v) {
  __builtin_nontemporal_store((_Float16)v, p + i);
}
__device__ __forceinline__ void stg4nt(GLB float* p, const float v[4]) {
  __builtin_nontemporal_store(vf4{v[0], v[1], v[2], v[3]}, reinterpret_cast<GLB vf4*>(p));
}
__device__ __forceinline__ void stg4nt(GLB _Float16* p, const float v[4]) {
  __builtin_nontemporal_store(vh4{(_Float16)v[0], (_Float16)v[1], (_Float16)v[2], (_Float16)v[3]},
                              reinterpret_cast<GLB vh4*>(p));
}

// Eight FP16 samples as one 16-byte streaming store: four dwords of packed halves (low
// half = lower column).
__device__ __forceinline__ uint32_t pack_h2(float a, float b) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)a) | ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)b) << 16);
}
__device__ __forceinline__ void stg8nt(GLB _Float16* p, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  typedef uint32_t vu4s __attribute__((ext_vector_type(4)));
  __builtin_nontemporal_store(vu4s{a, b, c, d}, reinterpret_cast<GLB vu4s*>(p));
}

__device__ __forceinline__ float ldv(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const _Float16* p, int64_t i) { return (float)p[i]; }
__device__ __forceinline__ void stv(float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void stv(_Float16* p, int64_t i, float v) { p[i] = (_Float16)v; }

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

// The same sequence from canvas coordinates already held as (exact) floats.
__device__ __forceinline__ void warp_coords_f(const float* __restrict__ h, float Xf, float Yf, float& x, float& y,
                                              bool& zpos) {
#pragma clang fp contract(off)
  const float u = (h[0] * Xf + h[1] * Yf) + h[2];
  const float v = (h[3] * Xf + h[4] * Yf) + h[5];
  const float z = (h[6] * Xf + h[7] * Yf) + h[8];
  zpos = z > 0.0f;
  x = u / z;
  y = v / z;
}

// The same sequence, also returning z.
__device__ __forceinline__ void warp_coords_z(const float* __restrict__ h, float Xf, float Yf, float& x, float& y,
                                              float& z) {
#pragma clang fp contract(off)
  const float u = (h[0] * Xf + h[1] * Yf) + h[2];
  const float v = (h[3] * Xf + h[4] * Yf) + h[5];
  z = (h[6] * Xf + h[7] * Yf) + h[8];
  x = u / z;
  y = v / z;
}

// x = u/z and y = v/z, correctly rounded, for operands in the range where the hardware
// division sequence scales nothing and fixes nothing up: z in [2^-10, 2^20] and |u|, |v|
// in [2^-12, 2^44] (exponent gaps far below 96, no denormal reciprocal, numerator or
// quotient).  In that range the IEEE divide of the
// compiler is exactly: r = rcp(z) refined by one Newton step, q = u r, two residual
// corrections; the refined reciprocal is shared by both quotients.
__device__ __forceinline__ void div2_in_range(float u, float v, float z, float& x, float& y) {
  float r = __builtin_amdgcn_rcpf(z);
  r = __builtin_fmaf(__builtin_fmaf(-z, r, 1.0f), r, r);
  float qx = u * r, qy = v * r;
  qx = __builtin_fmaf(__builtin_fmaf(-z, qx, u), r, qx);
  qy = __builtin_fmaf(__builtin_fmaf(-z, qy, v), r, qy);
  x = __builtin_fmaf(__builtin_fmaf(-z, qx, u), r, qx);
  y = __builtin_fmaf(__builtin_fmaf(-z, qy, v), r, qy);
}

// Eight bytes at any byte address (global memory accepts unaligned dword accesses).
typedef unsigned long long __attribute__((aligned(1))) u64_unaligned;
__device__ __forceinline__ unsigned long long ld8(const GLB uint8_t* p) { return *(const GLB u64_unaligned*)p; }

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
    if (cst(items)[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------------------------
// Fused pyramid pass from level k to k+1 (256 threads, four waves per workgroup).
//
// A tile is 64 level-k columns by 16 * sub rows; the workgroup walks down it in sub-steps
// of 16 rows.  Persistent, XCD-aware schedule: the tiles are split into eight contiguous
// ranges, one per XCD (workgroup b runs on XCD b % 8), and the workgroups of an XCD stride
// through its range, so neighbouring tiles -- which share halos -- share that XCD's L2.
//
// Stages of one sub-step:
//   A  (whole workgroup, then a barrier) stage the 71-column window of the sub-step's 23
//      rows (its 16 rows plus 4 above and 3 below) of every channel in LDS: three image
//      channels (the bilinear warp of the source frame at level 0, the stored G_k above)
//      and the seam weight.  LDS rows form a ring of 23: the 7 rows a sub-step shares with
//      the previous one stay where they are, so only its 16 new rows are staged (all 23 on
//      a tile's first sub-step).  At level 0 the source rectangle under a source-interior
//      window is first read into LDS as aligned 16-byte chunks (one more barrier) and the
//      bilinear taps come from there;
//   B..E  (wave w alone on channel slot w, no workgroup barrier)
//      B+C  REDUCE -> extended 34x10 coarse tile (horizontal then vertical in registers,
//           then into the wave's LDS rows); its interior, G_{k+1} / Gm_{k+1}, is stored
//           from LDS with one 16-byte store per lane;
//      D+E  horizontal and vertical EXPAND of the coarse tile and L_k = G_k - EXPAND(G_{k+1}),
//           stored on the band window (image channels only).
struct PyrTile {
  int item, X0, Y0, nsub;
};

__device__ __forceinline__ PyrTile decode_tile(const PyrItem* __restrict__ items, int nitems, int t) {
  PyrTile d;
  d.item = find_item(items, nitems, t);
  const CST PyrItem& it = cst(items)[d.item];
  const int lt = t - it.tile_begin;
  const int tyi = lt / it.tiles_x, txi = lt - tyi * it.tiles_x;
  d.X0 = it.tile_x0 + txi * kPyrTX;
  d.Y0 = it.tile_y0 + tyi * (kPyrTY * it.sub);
  d.nsub = min(it.sub, it.rows16 - tyi * it.sub);
  return d;
}

template <int N>
struct Rows {
  static constexpr int value = N;
};

template <typename T, bool EMIT_LAP, bool WARP>
__global__ void __launch_bounds__(kThreads, 4) k_pyr(const PyrItem* __restrict__ items, int nitems, int ntiles,
                                                     FrameArgs fa) {
  constexpr int TX = kPyrTX, TY = kPyrTY;
  constexpr int EW = TX + 7, EH = TY + 7;            // staged window: 4 before, 3 after
  constexpr int SW = 72;                             // LDS row strides are 16-byte multiples
  constexpr int CW = TX / 2 + 2, CH = TY / 2 + 2;    // coarse tile + one-sample halo
  // coarse tile of every channel: coarse column j at index j + 3, so the interior columns
  // 1 .. 32 start on a 16-byte boundary
  constexpr int HS = 40, CO = 3;
  __shared__ __attribute__((aligned(16))) float sIn[4][EH][SW];   // rows: ring
  __shared__ __attribute__((aligned(16))) float sC[4][CH][HS];
  // warp only: the rounded products h0 X, h3 X, h6 X of every staged column and h1 Y,
  // h4 Y, h7 Y of every window row, shared by the workgroup's samples
  constexpr int NCT = WARP ? EW : 1, NRT = WARP ? EH : 1;
  __shared__ __attribute__((aligned(16))) float sColT[NCT][4];
  __shared__ __attribute__((aligned(16))) float sRowT[NRT][4];
  // warp only: the class of every sub-step's 16-row window, classified together at the
  // tile's first sub-step (slot kMaxSub: the 7 rows that sub-step also stages)
  constexpr int kMaxSub = 8;
  __shared__ int sCls[kMaxSub + 1];
  // warp only: the source rectangle under a source-interior 16-row window, one 256-byte
  // LDS row per source row (read as aligned 16-byte chunks), and its origin
  constexpr int FH = 24, FWB = 256;
  static_assert(FWB == 256, "an LDS row of the source rectangle is 1 << 8 bytes");
  __shared__ __attribute__((aligned(16))) uint32_t sSrc[WARP ? FH : 1][FWB / 4];
  __shared__ int sBox[kMaxSub][4];   // per sub-step: bx0, by0, rows, 16-byte chunks per row
  constexpr uint32_t kPlaneRing = EH * SW * 4;       // bytes of one channel's ring of rows

  const int tid = threadIdx.x;
  // ---- schedule ----
  const int G = gridDim.x, b = blockIdx.x;
  int t, t_end, stride;
  if (G >= 8) {
    const int xcd = b & 7, rank = b >> 3;
    const int q = ntiles >> 3, r = ntiles & 7;
    const int t0 = xcd * q + min(xcd, r);
    t = t0 + rank;
    t_end = t0 + q + (xcd < r ? 1 : 0);
    stride = (G - xcd + 7) >> 3;
  } else {
    t = b;
    t_end = ntiles;
    stride = G;
  }

  for (; t < t_end; t += stride) {
    const PyrTile d = decode_tile(items, nitems, t);
    const CST PyrItem& it = cst(items)[d.item];
    const int X0 = d.X0;
    const int fw = it.fine_w, fh = it.fine_h;
    const int nimg = it.img_kind == kSrcNone ? 0 : it.nch;
    const bool has_mask = it.msk_kind != kSrcNone;
    const int nact = nimg + (has_mask ? 1 : 0);
    const int rx = it.roi_x, ry = it.roi_y, rw = it.roi_w, rh = it.roi_h;

    for (int s = 0; s < d.nsub; ++s) {
      const int Y0 = d.Y0 + s * TY;
      const int off = (s * TY) % EH;   // logical row r of the window lives in ring row (r + off) mod EH
      const uint32_t off4 = (uint32_t)off * (SW * 4);
      const bool interior = X0 >= 4 && X0 + TX + 3 <= fw && Y0 >= 4 && Y0 + TY + 3 <= fh;
      // stored levels of an interior window can be staged as aligned 16-byte chunks (above
      // level 0; see stage A)
      constexpr int kChunk = 16 / (int)sizeof(T);
      const bool chunked = !WARP && interior && rw > 0 && rh > 0 && ((X0 - rx) % kChunk) == 0 &&
                           (nimg == 0 || (((uintptr_t)it.img & 15) == 0 && (it.img_row % kChunk) == 0 &&
                                          (it.img_plane % kChunk) == 0)) &&
                           (!has_mask || (((uintptr_t)it.msk & 15) == 0 && (it.msk_row % kChunk) == 0));
      if (WARP) {
        // the coordinate tables (the columns once per tile, the rows per sub-step); their
        // last readers (the previous sub-step's stage A) finished before its closing barrier
        if (tid < EW) {
          if (s == 0) {
            const float Xf = (float)(X0 - 4 + tid);
            const float4 c = {it.hinv[0] * Xf, it.hinv[3] * Xf, it.hinv[6] * Xf, 0.0f};
            *reinterpret_cast<float4*>(sColT[tid]) = c;
          }
        } else if (tid >= 128 && tid < 128 + EH) {
          const float Yf = (float)(Y0 - 4 + (tid - 128));
          const float4 r = {it.hinv[1] * Yf, it.hinv[4] * Yf, it.hinv[7] * Yf, 0.0f};
          *reinterpret_cast<float4*>(sRowT[tid - 128]) = r;
        } else if (tid >= 192 && s == 0) {
          // Window classes of every sub-step of the tile, once per tile (wave 3; lanes
          // 8 u .. 8 u + 3: the corners of sub-step u's 16 new rows, lanes 4-7: of the 7
          // rows the first sub-step also stages).
          // Source-interior (bit 0): z > 0 at the four corners (so on all of the window: z
          // is affine) and their source positions inside [1, w-3) x [1, h-2).  The map is
          // projective there, so every staged sample lies in the convex hull of the corner
          // images (up to FP32 rounding, far below the one-sample margin): its four taps
          // are in the frame and the pair of taps of a row is one 8-byte read that ends
          // inside the row.  Source-exterior (bit 1): z > 0 at the corners and all four
          // corner images at least one sample beyond the same side of the frame (x <= -2,
          // x >= w + 1, y <= -2 or y >= h + 1): every staged sample's taps are outside,
          // its G_0 is 0.  Either also needs the window inside the canvas (checked by the
          // stage).
          const int lane = tid - 192, u = lane >> 3, j = lane & 7;
          const int nsc = min(d.nsub, kMaxSub);
          bool bad = false, zok = false, lft = false, rgt = false, top = false, bot = false;
          float xc = 0.0f, yc = 0.0f;
          const int w = it.frame_w, h = it.frame_h;
          if (u < nsc && (j < 4 || u == 0)) {
            float hv[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) hv[i] = it.hinv[i];
            const int r0 = j < 4 ? EH - TY : 0, r1 = j < 4 ? EH - 1 : EH - TY - 1;
            float zc;
            warp_coords_z(hv, (float)(X0 - 4 + ((j & 1) ? EW - 1 : 0)),
                          (float)(d.Y0 + u * TY - 4 + ((j & 2) ? r1 : r0)), xc, yc, zc);
            zok = zc >= 0x1p-10f && zc <= 0x1p20f;
            bad = !(zok && xc >= 1.0f && xc < (float)(w - 3) && yc >= 1.0f && yc < (float)(h - 2));
            lft = xc <= -2.0f;
            rgt = xc >= (float)(w + 1);
            top = yc <= -2.0f;
            bot = yc >= (float)(h + 1);
          }
          const uint64_t mb = __ballot(bad), mz = __ballot(zok), ml = __ballot(lft), mr = __ballot(rgt),
                         mt = __ballot(top), mo = __ballot(bot);
          // bounding box of each group of four corner images
          float mnx = xc, mxx = xc, mny = yc, mxy = yc;
#pragma unroll
          for (int dd = 1; dd < 4; dd <<= 1) {
            mnx = fminf(mnx, __shfl_xor(mnx, dd));
            mxx = fmaxf(mxx, __shfl_xor(mxx, dd));
            mny = fminf(mny, __shfl_xor(mny, dd));
            mxy = fmaxf(mxy, __shfl_xor(mxy, dd));
          }
          if (u < nsc && (j == 0 || (j == 4 && u == 0))) {
            const int sh = lane;
            auto all4 = [sh](uint64_t m) { return ((m >> sh) & 15ull) == 15ull; };
            const bool fast = ((mb >> sh) & 15ull) == 0ull;
            const bool outside = all4(mz) && (all4(ml) || all4(mr) || all4(mt) || all4(mo));
            // Staged (bit 2, 16-row windows only): every tap lies in the box [bx0, bx1] x
            // [by0, by1] (the corner images' bounding box, one sample wider on each side
            // for rounding), which fits the LDS rows, and the 16-byte chunks covering a
            // box row (from its start rounded down to 16 bytes, at most 15 + 3 nbx + 15
            // bytes) stay inside the frame row: bx0 >= 5 and bx1 <= w - 11.  The row
            // pitch is a multiple of 16 bytes, so every box row starts at the same offset
            // in its LDS row.
            bool staged = false;
            const int64_t srow = fa.n ? fa.row[it.frame_slot] : it.img_row;
            if (j == 0 && fast && (srow & 15) == 0) {
              const int bx0 = (int)floorf(mnx) - 1, bx1 = (int)floorf(mxx) + 2;
              const int by0 = (int)floorf(mny) - 1, by1 = (int)floorf(mxy) + 2;
              const int nbx = bx1 - bx0 + 1, nby = by1 - by0 + 1;
              staged = bx0 >= 5 && bx1 <= w - 11 && by0 >= 0 && by1 <= h - 1 && 15 + 3 * nbx <= FWB && nby <= FH;
              if (staged) {
                sBox[u][0] = bx0;
                sBox[u][1] = by0;
                sBox[u][2] = nby;
                sBox[u][3] = (15 + 3 * nbx + 15) / 16;
              }
            }
            sCls[j == 0 ? u : kMaxSub] = (fast ? 1 : 0) | (outside ? 2 : 0) | (staged ? 4 : 0);
          }
        }
      }
      __syncthreads();   // the previous sub-step's readers of LDS are done

      // ---- A: stage logical rows R0 .. R0+NR-1 ----
      auto stage_a = [&](auto rows_c, auto r0_c) __attribute__((always_inline)) {
        constexpr int NR = decltype(rows_c)::value;
        constexpr int R0 = decltype(r0_c)::value;
        constexpr int NE = NR * EW;
        constexpr int NQ = (NE + kThreads - 1) / kThreads;
        // recomputed per sub-step (cheap) rather than held in registers across the loop
        int tid_l = tid;
        asm volatile("" : "+v"(tid_l));
        int rr[NQ], cc[NQ];                       // logical row (-1: idle slot) and column
        uint32_t lo[NQ];                          // byte offset of the slot in a channel's rows, unrotated
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int e = tid_l + q * kThreads;
          rr[q] = e < NE ? R0 + e / EW : -1;
          cc[q] = e < NE ? e % EW : 0;
          // idle slots write the padding column EW (read by stage B's last float4 but never
          // used), so stores need no branch and loads are never sunk into one
          lo[q] = (uint32_t)((rr[q] < 0 ? R0 : rr[q]) * SW + (rr[q] < 0 ? EW : cc[q])) * 4u;
        }
        // When the stage's samples end inside its last round of slots, that round is idle
        // for whole waves (the 16-row stage: the waves of threads 128 .. 255); they skip it.
        const bool last_live = NE % kThreads == 0 || __builtin_amdgcn_readfirstlane(tid >> 6) * 64 + (NQ - 1) * kThreads < NE;
        auto live = [&](int q) { return q < NQ - 1 || last_live; };
        // the slot's cell in channel plane ch, rotated into the ring
        auto cell = [&](int ch, int q) -> float& {
          const uint32_t a = lo[q] + off4;
          return *reinterpret_cast<float*>(reinterpret_cast<char*>(&sIn[ch][0][0]) + min(a, a - kPlaneRing));
        };
        // canvas position of a slot (idle slots take the window's first sample)
        auto canvas = [&](int q, int& X, int& Y) {
          X = X0 - 4 + cc[q];
          Y = Y0 - 4 + (rr[q] < 0 ? R0 : rr[q]);
          if (!interior) {
            X = fold(X, fw);
            Y = fold(Y, fh);
          }
        };
        if (WARP) {
          const GLB uint8_t* src = cg<uint8_t>(fa.n ? (const void*)fa.ptr[it.frame_slot] : it.img);
          const int64_t srow = fa.n ? fa.row[it.frame_slot] : it.img_row;
          const int w = it.frame_w, h = it.frame_h;
          float hv[9];
#pragma unroll
          for (int i = 0; i < 9; ++i) hv[i] = it.hinv[i];
          const uint32_t srow32 = (uint32_t)srow;
          // seam weights (uint8 on the ROI, 0 outside): read first, used last
          const GLB uint8_t* msk = cg<uint8_t>(it.msk);
          uint32_t mv[NQ];
          const bool inside = interior && X0 - 4 >= rx && X0 + TX + 3 <= rx + rw && Y0 - 4 + R0 >= ry &&
                              Y0 - 4 + R0 + NR <= ry + rh;
          if (has_mask && inside) {
            const GLB uint8_t* m0 = msk + (int64_t)(Y0 - 4 + R0 - ry) * it.msk_row + (X0 - 4 - rx);
            const uint32_t mrow = (uint32_t)it.msk_row;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
              if (live(q)) mv[q] = m0[__umul24((uint32_t)(rr[q] < 0 ? 0 : rr[q] - R0), mrow) + (uint32_t)cc[q]];
          } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (!live(q)) continue;
              int X, Y;
              canvas(q, X, Y);
              const int my = Y - ry, mx = X - rx;
              const bool in = has_mask && my >= 0 && my < rh && mx >= 0 && mx < rw;
              const uint32_t m = has_mask ? (uint32_t)msk[in ? (int64_t)my * it.msk_row + mx : 0] : 0u;
              mv[q] = in ? m : 0u;
            }
          }
          const float fwf = (float)w, fhf = (float)h, fwm1 = (float)(w - 1), fhm1 = (float)(h - 1);
          // the window's class, computed before the sub-step's barrier
          const int cls = !interior ? 0 : R0 == 0 ? sCls[kMaxSub] : s < kMaxSub ? sCls[s] : 0;
          const bool fast = (cls & 1) != 0, outside = (cls & 2) != 0;
          if (outside) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (!live(q)) continue;
              cell(0, q) = 0.0f;
              cell(1, q) = 0.0f;
              cell(2, q) = 0.0f;
              cell(3, q) = (float)mv[q] * kInv255;
            }
          } else if (fast && (cls & 4) != 0) {
            // Source rectangle staged in LDS: its rows are read as aligned 16-byte chunks
            // (the reads of the whole workgroup cover it once), each sample's coordinates
            // are computed meanwhile, and its two 8-byte tap pairs come from LDS.
            const int bx0 = sBox[s][0], by0 = sBox[s][1], nby = sBox[s][2], nck = sBox[s][3];
            constexpr int NCK = (FH * (FWB / 16) + kThreads - 1) / kThreads;
            typedef uint32_t vu4 __attribute__((ext_vector_type(4)));
            vu4 ck[NCK];
#pragma unroll
            for (int k = 0; k < NCK; ++k) {
              // spare lanes repeat a chunk of the box (the same bytes to the same place)
              const int e = tid + k * kThreads, r = min(e / (FWB / 16), nby - 1), c = min(e % (FWB / 16), nck - 1);
              const uintptr_t a = ((uintptr_t)src + __umul24((uint32_t)(by0 + r), srow32) + 3u * (uint32_t)bx0) & ~(uintptr_t)15;
              ck[k] = *reinterpret_cast<const GLB vu4*>(a + 16u * (uint32_t)c);
            }
            // every box row starts in its LDS row at byte (frame address of the box row) mod 16
            const uint32_t s1 = ((uint32_t)(uintptr_t)src + 3u * (uint32_t)bx0) & 15u;
            float fxq[NQ], fyq[NQ];
            uint32_t o1[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (!live(q)) continue;
              // the coordinate sequence from the tabled products (the same roundings as
              // the direct one; the in-range division is the IEEE one)
              const float4 ct = *reinterpret_cast<const float4*>(sColT[cc[q]]);
              const float4 rt = *reinterpret_cast<const float4*>(sRowT[rr[q] < 0 ? R0 : rr[q]]);
              float u, v, z, x, y;
              {
#pragma clang fp contract(off)
                u = (ct.x + rt.x) + hv[2];
                v = (ct.y + rt.y) + hv[5];
                z = (ct.z + rt.z) + hv[8];
              }
              div2_in_range(u, v, z, x, y);
              fxq[q] = __builtin_amdgcn_fractf(x);
              fyq[q] = __builtin_amdgcn_fractf(y);
              const uint32_t xi = (uint32_t)(int)x, yi = (uint32_t)(int)y;
              // 24-bit multiplies (full rate): the box is under 256 samples wide and 24 rows
              const uint32_t r = yi - (uint32_t)by0, dx = __umul24(xi - (uint32_t)bx0, 3u);
              o1[q] = (r << 8) + s1 + dx;
            }
#pragma unroll
            for (int k = 0; k < NCK; ++k) {
              const int e = tid + k * kThreads, r = min(e / (FWB / 16), nby - 1), c = min(e % (FWB / 16), nck - 1);
              *reinterpret_cast<vu4*>(&sSrc[r][4 * c]) = ck[k];
            }
            __syncthreads();
            const uint8_t* sb = reinterpret_cast<const uint8_t*>(&sSrc[0][0]);
            auto ld8s = [&](uint32_t o) -> unsigned long long {
              const uint32_t* d = reinterpret_cast<const uint32_t*>(sb + (o & ~3u));
              const uint32_t w0 = d[0], w1 = d[1], w2 = d[2];
              const uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, o & 3u);
              const uint32_t hi = __builtin_amdgcn_alignbyte(w2, w1, o & 3u);
              return (unsigned long long)lo | ((unsigned long long)hi << 32);
            };
            // every sample's tap reads first, then the bilinear combination
            unsigned long long ras[NQ], rbs[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (!live(q)) continue;
              ras[q] = ld8s(o1[q]);
              rbs[q] = ld8s(o1[q] + FWB);
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (!live(q)) continue;
              const unsigned long long ra = ras[q], rb = rbs[q];
              const float fx = fxq[q], fy = fyq[q], gx = 1.0f - fx, gy = 1.0f - fy;
              const float gyi = gy * kInv255, fyi = fy * kInv255;
              const float w00 = gyi * gx, w01 = gyi * fx, w10 = fyi * gx, w11 = fyi * fx;
              const uint32_t a0 = (uint32_t)ra, a1 = (uint32_t)(ra >> 32);
              const uint32_t b0 = (uint32_t)rb, b1 = (uint32_t)(rb >> 32);
              const float p00[3] = {(float)(a0 & 255u), (float)((a0 >> 8) & 255u), (float)((a0 >> 16) & 255u)};
              const float p01[3] = {(float)(a0 >> 24), (float)(a1 & 255u), (float)((a1 >> 8) & 255u)};
              const float p10[3] = {(float)(b0 & 255u), (float)((b0 >> 8) & 255u), (float)((b0 >> 16) & 255u)};
              const float p11[3] = {(float)(b0 >> 24), (float)(b1 & 255u), (float)((b1 >> 8) & 255u)};
#pragma unroll
              for (int ch = 0; ch < 3; ++ch)
                cell(ch, q) = w00 * p00[ch] + w01 * p01[ch] + w10 * p10[ch] + w11 * p11[ch];
              cell(3, q) = (float)mv[q] * kInv255;
            }
          } else if (fast) {
            // every sample: coordinates and both row reads issued first, so a wave keeps
            // 2 * NQ reads in flight; then the bilinear combination
            unsigned long long ra[NQ], rb[NQ];
            float fxq[NQ], fyq[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (!live(q)) continue;
              // z lies between its corner values and x, y in [1, w) x [1, h): the in-range
              // division is the IEEE one, x - floor(x) is exact and truncation is floor
              // the coordinate sequence from the tabled products (the same roundings)
              const float4 ct = *reinterpret_cast<const float4*>(sColT[cc[q]]);
              const float4 rt = *reinterpret_cast<const float4*>(sRowT[rr[q] < 0 ? R0 : rr[q]]);
              float u, v, z, x, y;
              {
#pragma clang fp contract(off)
                u = (ct.x + rt.x) + hv[2];
                v = (ct.y + rt.y) + hv[5];
                z = (ct.z + rt.z) + hv[8];
              }
              div2_in_range(u, v, z, x, y);
              fxq[q] = __builtin_amdgcn_fractf(x);
              fyq[q] = __builtin_amdgcn_fractf(y);
              const uint32_t o = __umul24((uint32_t)(int)y, srow32) + __umul24((uint32_t)(int)x, 3u);
              ra[q] = ld8(src + o);
              rb[q] = ld8(src + (o + srow32));
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (!live(q)) continue;
              const float fx = fxq[q], fy = fyq[q], gx = 1.0f - fx, gy = 1.0f - fy;
              const float gyi = gy * kInv255, fyi = fy * kInv255;
              const float w00 = gyi * gx, w01 = gyi * fx, w10 = fyi * gx, w11 = fyi * fx;
              const uint32_t a0 = (uint32_t)ra[q], a1 = (uint32_t)(ra[q] >> 32);
              const uint32_t b0 = (uint32_t)rb[q], b1 = (uint32_t)(rb[q] >> 32);
              const float p00[3] = {(float)(a0 & 255u), (float)((a0 >> 8) & 255u), (float)((a0 >> 16) & 255u)};
              const float p01[3] = {(float)(a0 >> 24), (float)(a1 & 255u), (float)((a1 >> 8) & 255u)};
              const float p10[3] = {(float)(b0 & 255u), (float)((b0 >> 8) & 255u), (float)((b0 >> 16) & 255u)};
              const float p11[3] = {(float)(b0 >> 24), (float)(b1 & 255u), (float)((b1 >> 8) & 255u)};
#pragma unroll
              for (int ch = 0; ch < 3; ++ch)
                cell(ch, q) = w00 * p00[ch] + w01 * p01[ch] + w10 * p10[ch] + w11 * p11[ch];
              cell(3, q) = (float)mv[q] * kInv255;
            }
          } else {
            // General window (frame borders, canvas edges): taps outside the frame weigh
            // 0.  Each row pair is still one 8-byte read, from a start clamped into
            // [0, 3w - 8] of a row clamped into the frame (w >= 3), so no read leaves its
            // row; the pair is shifted into place afterwards.
            unsigned long long ra[NQ], rb[NQ];
            float fxq[NQ], fyq[NQ];
            uint32_t tapq[NQ];                   // bits: 00 01 10 11 inside, << 4: byte shift + 3
            const uint32_t lastc = 3u * (uint32_t)w - 8u;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (!live(q)) continue;
              int Xc, Yc;
              canvas(q, Xc, Yc);
              float x, y;
              bool zpos;
              warp_coords_f(hv, (float)Xc, (float)Yc, x, y, zpos);
              const bool ok = zpos && x >= -1.0f && x < fwf && y >= -1.0f && y < fhf;
              const float xs = ok ? x : 0.0f, ys = ok ? y : 0.0f;
              const float x0f = floorf(xs), y0f = floorf(ys);
              fxq[q] = xs - x0f;
              fyq[q] = ys - y0f;
              const bool xa = ok && x0f >= 0.0f, xb = ok && x0f < fwm1, ya = y0f >= 0.0f, yb = y0f < fhm1;
              const int x0 = (int)x0f, y0 = (int)y0f;              // x0 >= -1, y0 >= -1
              const int c3 = 3 * x0;
              const uint32_t start = (uint32_t)min(max(c3, 0), (int)lastc);
              const uint32_t r0 = (uint32_t)max(y0, 0), r1 = (uint32_t)min(y0 + 1, h - 1);
              tapq[q] = (uint32_t)(ya && xa) | ((uint32_t)(ya && xb) << 1) | ((uint32_t)(yb && xa) << 2) |
                        ((uint32_t)(yb && xb) << 3) | ((uint32_t)(c3 - (int)start + 3) << 4);
              ra[q] = ld8(src + (__umul24(r0, srow32) + start));
              rb[q] = ld8(src + (__umul24(r1, srow32) + start));
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (!live(q)) continue;
              const int sh = (int)(tapq[q] >> 4) - 3;              // byte offset of tap 0: -3 .. 5
              const unsigned long long a = sh >= 0 ? ra[q] >> (8 * sh) : ra[q] << 24;
              const unsigned long long bq = sh >= 0 ? rb[q] >> (8 * sh) : rb[q] << 24;
              const float fx = fxq[q], fy = fyq[q], gx = 1.0f - fx, gy = 1.0f - fy;
              const float gyi = gy * kInv255, fyi = fy * kInv255;
              const uint32_t tp = tapq[q];
              const float w00 = (tp & 1u) ? gyi * gx : 0.0f, w01 = (tp & 2u) ? gyi * fx : 0.0f;
              const float w10 = (tp & 4u) ? fyi * gx : 0.0f, w11 = (tp & 8u) ? fyi * fx : 0.0f;
              const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
              const uint32_t b0 = (uint32_t)bq, b1 = (uint32_t)(bq >> 32);
              const float p00[3] = {(float)(a0 & 255u), (float)((a0 >> 8) & 255u), (float)((a0 >> 16) & 255u)};
              const float p01[3] = {(float)(a0 >> 24), (float)(a1 & 255u), (float)((a1 >> 8) & 255u)};
              const float p10[3] = {(float)(b0 & 255u), (float)((b0 >> 8) & 255u), (float)((b0 >> 16) & 255u)};
              const float p11[3] = {(float)(b0 >> 24), (float)(b1 & 255u), (float)((b1 >> 8) & 255u)};
#pragma unroll
              for (int ch = 0; ch < 3; ++ch)
                cell(ch, q) = w00 * p00[ch] + w01 * p01[ch] + w10 * p10[ch] + w11 * p11[ch];
              cell(3, q) = (float)mv[q] * kInv255;
            }
          }
        } else if (chunked) {
          // Stored G_k planes and Gm_k on the ROI (0 outside) as aligned 16-byte chunks of C
          // samples: window row r of channel slot c is chunks k = 0 .. NCH-1 of plane row
          // Y0 - 4 + R0 + r - ry from plane column X0 - C - rx + C k (the tile's X0 - rx, the
          // row pitches and plane strides are multiples of C, the planes start on 16-byte
          // boundaries, and a row's pitch covers its width rounded up to C).  Every read is
          // issued, without a branch, from a chunk clamped into the plane (its row into
          // [0, rh), its column into the rounded width); samples outside the ROI, the
          // channel set or the window are dropped afterwards.
          constexpr int C = 16 / (int)sizeof(T);
          constexpr int NCH = 64 / C + 2;
          constexpr int NT = NR * 4 * NCH;
          constexpr int NQC = (NT + kThreads - 1) / kThreads;
          typedef uint32_t vu4c __attribute__((ext_vector_type(4)));
          const int rwc = (rw + C - 1) / C;
          const int k0 = (X0 - C - rx) / C;   // plane chunk of k = 0
          // the descriptor's fields once, as scalars (a per-lane choice between two fields
          // would read them per lane and wait for each)
          const GLB T* const gimg = cg<T>(it.img);
          const GLB T* const gmsk = cg<T>(it.msk);
          const uint32_t iplane = (uint32_t)it.img_plane, irow = (uint32_t)it.img_row, mrow = (uint32_t)it.msk_row;
          uint32_t raw[NQC][4];   // plain dwords: an array of 4-vectors lost its upper elements at NQC = 5
#pragma unroll
          for (int q = 0; q < NQC; ++q) {
            const int e = min(tid_l + q * kThreads, NT - 1);
            const int k = e % NCH, rest = e / NCH, slot = rest & 3, r = rest >> 2;
            const bool from_img = slot < 3 ? nimg > 0 : !has_mask;
            const GLB T* base = from_img ? gimg + (uint32_t)min(slot, max(nimg - 1, 0)) * iplane : gmsk;
            const uint32_t pitch = from_img ? irow : mrow;
            const int prow = min(max(Y0 - 4 + R0 + r - ry, 0), rh - 1);
            const int pck = min(max(k0 + k, 0), rwc - 1);
            const vu4c t = *reinterpret_cast<const GLB vu4c*>(base + (__umul24((uint32_t)prow, pitch) + (uint32_t)(C * pck)));
            raw[q][0] = t.x;
            raw[q][1] = t.y;
            raw[q][2] = t.z;
            raw[q][3] = t.w;
          }
#pragma unroll
          for (int q = 0; q < NQC; ++q) {
            const int e = tid_l + q * kThreads;
            if (e >= NT) continue;
            const int k = e % NCH, rest = e / NCH, slot = rest & 3, r = rest >> 2;
            const int prow = Y0 - 4 + R0 + r - ry, c0 = C * (k0 + k);
            const bool ok = (slot < 3 ? slot < nimg : has_mask) && prow >= 0 && prow < rh;
            const int keep = ok ? min(max(rw - c0, 0), (c0 < 0 ? 0 : C)) : 0;   // leading samples kept
            float v[C];
#pragma unroll
            for (int i = 0; i < C; ++i) {
              const float smp = sizeof(T) == 4 ? __builtin_bit_cast(float, raw[q][i & 3])
                                               : from_raw((uint16_t)(raw[q][i >> 1] >> (16 * (i & 1))));
              v[i] = i < keep ? smp : 0.0f;
            }
            // window column of v[0], a multiple of 4; only columns 0 .. SW-1 exist
            const int wc = C * k - C + 4;
            const uint32_t a0 = (uint32_t)((R0 + r) * SW) * 4u + off4;
            char* rowb = reinterpret_cast<char*>(&sIn[slot][0][0]) + min(a0, a0 - kPlaneRing);
#pragma unroll
            for (int h = 0; h < C / 4; ++h) {
              const int col = wc + 4 * h;
              if (col >= 0 && col < SW)
                *reinterpret_cast<float4*>(rowb + 4 * col) = float4{v[4 * h], v[4 * h + 1], v[4 * h + 2], v[4 * h + 3]};
            }
          }
        } else {
          // stored G_k planes and Gm_k on the ROI (0 outside): every read is issued first, as
          // raw bits from an address inside the planes (channel clamped to the last plane,
          // offset 0 outside the ROI); conversion and zeroing come afterwards
          const GLB T* g = cg<T>(nimg > 0 ? it.img : it.msk);
          const int64_t grow = nimg > 0 ? it.img_row : it.msk_row, gplane = nimg > 0 ? it.img_plane : 0;
          const GLB T* m = has_mask ? cg<T>(it.msk) : g;
          const int64_t mrow = has_mask ? it.msk_row : grow;
          const int cmax = nimg > 0 ? nimg - 1 : 0;
          typename RawOf<T>::type raw[NQ][4];
          bool inq[NQ];
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if (!live(q)) continue;
            int X, Y;
            canvas(q, X, Y);
            Y -= ry;
            X -= rx;
            inq[q] = X >= 0 && X < rw && Y >= 0 && Y < rh;
            const uint32_t og = inq[q] ? __umul24((uint32_t)Y, (uint32_t)grow) + (uint32_t)X : 0u;
            const uint32_t om = inq[q] ? __umul24((uint32_t)Y, (uint32_t)mrow) + (uint32_t)X : 0u;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) raw[q][ch] = ld_raw(g, (uint32_t)min(ch, cmax) * (uint32_t)gplane + og);
            raw[q][3] = ld_raw(m, om);
          }
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if (!live(q)) continue;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) cell(ch, q) = (inq[q] && ch < nimg) ? from_raw(raw[q][ch]) : 0.0f;
            cell(3, q) = (inq[q] && has_mask) ? from_raw(raw[q][3]) : 0.0f;
          }
        }
      };
      // a tile's first sub-step also stages the 7 rows the ring would otherwise carry over
      if (s == 0) stage_a(Rows<EH - TY>(), Rows<0>());
      stage_a(Rows<TY>(), Rows<EH - TY>());
      __syncthreads();

      // ---- B..E: wave w works on channel slot w alone, and exchanges data only through
      //      its own LDS rows (sC[ch]), so the next workgroup barrier is the next sub-step's ----
      const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
      const int lane = tid & 63;
      if (wv >= nact) continue;
      // With all four channels, the mask (whose wave has no D+E) goes to wave s & 1: a
      // workgroup's waves run on the compute unit's four SIMDs one each, and waves 0 and 1
      // also took stage A's last, partial round of samples, so every SIMD gets about the
      // same arithmetic per two sub-steps.
      const int mw = s & 1;
      const int ch = nact == 4 && nimg == 3 ? (wv == mw ? 3 : wv - (wv > mw ? 1 : 0)) : (wv < nimg ? wv : 3);
      // logical row r of the channel's ring (byte offsets keep the arithmetic 32-bit)
      const char* plane = reinterpret_cast<const char*>(&sIn[ch][0][0]);
      auto rowp = [&](int r) -> const float* {
        const uint32_t a = (uint32_t)r * (SW * 4) + off4;
        return reinterpret_cast<const float*>(plane + min(a, a - kPlaneRing));
      };
      // B+C: REDUCE -> extended coarse tile (CH x CW with a one-sample halo) in sC[ch].
      // Lane (g, jp), g < 3: coarse columns 2jp, 2jp+1 of coarse rows 3g .. 3g+3, from the
      // eleven fine rows 6g .. 6g+10, each reduced horizontally from two b128 reads; rows 3
      // and 6 are written by the group that starts there.
      if (lane < 3 * (CW / 2)) {
        const int g = lane / (CW / 2), jp = lane - (CW / 2) * g, rs = 3 * g;
        float2 hr[11];
#pragma unroll
        for (int u = 0; u < 11; ++u) {
          const float* row = rowp(2 * rs + u) + 4 * jp;
          const float4 a = *reinterpret_cast<const float4*>(row);
          const float4 bq = *reinterpret_cast<const float4*>(row + 4);
          hr[u].x = kW0 * (a.x + bq.x) + kW1 * (a.y + a.w) + kW2 * a.z;
          hr[u].y = kW0 * (a.z + bq.z) + kW1 * (a.w + bq.y) + kW2 * bq.x;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if (m == 0 && g > 0) continue;
          float2 o;
          o.x = kW0 * (hr[2 * m].x + hr[2 * m + 4].x) + kW1 * (hr[2 * m + 1].x + hr[2 * m + 3].x) +
                kW2 * hr[2 * m + 2].x;
          o.y = kW0 * (hr[2 * m].y + hr[2 * m + 4].y) + kW1 * (hr[2 * m + 1].y + hr[2 * m + 3].y) +
                kW2 * hr[2 * m + 2].y;
          float* c = &sC[ch][rs + m][CO + 2 * jp];
          c[0] = o.x;
          c[1] = o.y;
        }
      }
      // the wave's own sC[ch] rows: LDS accesses of one wave complete in order
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // the interior (8 x 32) is G_{k+1} / Gm_{k+1}: lane (i, m) stores coarse row 1 + i,
      // columns 1 + 4m .. 4 + 4m, one 16-byte store where the four are inside the coarse ROI
      {
        const int i = 1 + (lane >> 3), j = 1 + 4 * (lane & 7);
        const float4 v4 = *reinterpret_cast<const float4*>(&sC[ch][i][CO + j]);
        const float v[4] = {v4.x, v4.y, v4.z, v4.w};
        const int cy = Y0 / 2 - 1 + i - it.croi_y, cx = X0 / 2 - 1 + j - it.croi_x;
        // FP16: lanes 2m and 2m+1 hold eight adjacent samples; the even lane stores all
        // eight as one 16-byte vector (the partner's four halves come by a lane swap)
        uint32_t h01 = 0, h23 = 0, p01 = 0, p23 = 0;
        if (sizeof(T) == 2) {
          h01 = pack_h2(v[0], v[1]);
          h23 = pack_h2(v[2], v[3]);
          p01 = __shfl_xor(h01, 1);
          p23 = __shfl_xor(h23, 1);
        }
        if (cy >= 0 && cy < it.croi_h) {
          GLB T* out = ch < 3 ? mg<T>(it.g_out) : mg<T>(it.gm_out);
          // 32-bit element offsets (the host keeps every level's planes under 2^31
          // elements and its rows under 2^23)
          const uint32_t orow = (uint32_t)(ch < 3 ? it.g_row : it.gm_row);
          const uint32_t obase = ch < 3 ? (uint32_t)ch * (uint32_t)it.g_plane : 0u;
          const int ob = (int)(obase + __umul24((uint32_t)cy, orow)) + cx;
          const bool odd = (lane & 1) != 0;
          const int cxe = cx - (odd ? 4 : 0), obe = ob - (odd ? 4 : 0);
          if (sizeof(T) == 2 && cxe >= 0 && cxe + 7 < it.croi_w && ((uintptr_t)(out + obe) & 15) == 0) {
            if (!odd) stg8nt(reinterpret_cast<GLB _Float16*>(out + obe), h01, h23, p01, p23);
          } else if (cx >= 0 && cx + 3 < it.croi_w && ((uintptr_t)(out + ob) & (4 * sizeof(T) - 1)) == 0) {
            stg4nt(out + ob, v);
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (cx + u >= 0 && cx + u < it.croi_w) stgnt(out, ob + u, v[u]);
          }
        }
      }
      if (!EMIT_LAP || ch == 3) continue;
      const bool lap_tile = it.lw_w > 0 && X0 < it.lw_x + it.lw_w && X0 + TX > it.lw_x &&
                            Y0 < it.lw_y + it.lw_h && Y0 + TY > it.lw_y;
      if (!lap_tile) continue;

      // D+E: lane (rq, mm): fine columns 4mm .. 4mm+3 of fine rows 4rq .. 4rq+3.  Horizontal
      // EXPAND of coarse rows 2rq .. 2rq+3, then vertical EXPAND and the band
      // L_k = G_k - EXPAND(G_{k+1}), stored on the band window.
      {
        const int mm = lane & 15, rq = lane >> 4, x = 4 * mm;
        float4 eh[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float* c = &sC[ch][2 * rq + k][CO + 2 * mm];
          const float2 lo = {c[0], c[1]}, hi = {c[2], c[3]};
          eh[k].x = 0.125f * (lo.x + hi.x) + 0.75f * lo.y;
          eh[k].y = 0.5f * (lo.y + hi.x);
          eh[k].z = 0.125f * (lo.y + hi.y) + 0.75f * hi.x;
          eh[k].w = 0.5f * (hi.x + hi.y);
        }
        const int X = X0 + x - it.lw_x;
        GLB T* lout = mg<T>(it.l_out);
        float l[4][4];
#pragma unroll
        for (int yy = 0; yy < 4; ++yy) {
          const int y = 4 * rq + yy, k = yy >> 1;
          float4 ev;
          if (yy & 1) {
            ev.x = 0.5f * (eh[k + 1].x + eh[k + 2].x); ev.y = 0.5f * (eh[k + 1].y + eh[k + 2].y);
            ev.z = 0.5f * (eh[k + 1].z + eh[k + 2].z); ev.w = 0.5f * (eh[k + 1].w + eh[k + 2].w);
          } else {
            ev.x = 0.125f * (eh[k].x + eh[k + 2].x) + 0.75f * eh[k + 1].x;
            ev.y = 0.125f * (eh[k].y + eh[k + 2].y) + 0.75f * eh[k + 1].y;
            ev.z = 0.125f * (eh[k].z + eh[k + 2].z) + 0.75f * eh[k + 1].z;
            ev.w = 0.125f * (eh[k].w + eh[k + 2].w) + 0.75f * eh[k + 1].w;
          }
          const float4 gv = *reinterpret_cast<const float4*>(rowp(y + 4) + x + 4);
          l[yy][0] = gv.x - ev.x; l[yy][1] = gv.y - ev.y; l[yy][2] = gv.z - ev.z; l[yy][3] = gv.w - ev.w;
        }
        // FP16: lanes 2m and 2m+1 hold eight adjacent columns of the same four rows; the
        // even lane stores rows 0-1 and the odd lane rows 2-3 as 16-byte vectors, each
        // taking the partner's halves of those rows by a lane swap
        const bool odd = (mm & 1) != 0;
        const int Xe = X - (odd ? 4 : 0);
        bool pair = false;
        uint32_t own[2][2] = {}, oth[2][2] = {};
        if (sizeof(T) == 2) {
          uint32_t hp[4][2];
#pragma unroll
          for (int yy = 0; yy < 4; ++yy) {
            hp[yy][0] = pack_h2(l[yy][0], l[yy][1]);
            hp[yy][1] = pack_h2(l[yy][2], l[yy][3]);
          }
#pragma unroll
          for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
            for (int w2 = 0; w2 < 2; ++w2) {
              // send the rows the partner stores, keep the ones this lane stores
              own[r2][w2] = odd ? hp[2 + r2][w2] : hp[r2][w2];
              oth[r2][w2] = __shfl_xor(odd ? hp[r2][w2] : hp[2 + r2][w2], 1);
            }
          pair = Xe >= 0 && Xe + 7 < it.lw_w && ((uintptr_t)(lout + Xe) & 15) == 0 &&
                 ((it.l_row | it.l_plane) & 7) == 0;
        }
#pragma unroll
        for (int yy = 0; yy < 4; ++yy) {
          const int y = 4 * rq + yy;
          const int Y = Y0 + y - it.lw_y;
          const bool rowin = Y >= 0 && Y < it.lw_h;
          if (sizeof(T) == 2 && pair) {
            // this lane's two rows (the even lane's 0-1, the odd lane's 2-3)
            if (yy < 2) {
              const int Ys = Y + (odd ? 2 : 0);
              if (Ys >= 0 && Ys < it.lw_h) {
                const int base = ch * (int)it.l_plane + __mul24(Ys, (int)it.l_row) + Xe;
                GLB _Float16* q = reinterpret_cast<GLB _Float16*>(lout + base);
                if (odd) stg8nt(q, oth[yy][0], oth[yy][1], own[yy][0], own[yy][1]);
                else stg8nt(q, own[yy][0], own[yy][1], oth[yy][0], oth[yy][1]);
              }
            }
            continue;
          }
          const bool full = rowin && X >= 0 && X + 3 < it.lw_w;
          const int base = ch * (int)it.l_plane + __mul24(Y, (int)it.l_row) + X;
          if (full && ((uintptr_t)(lout + base) & (4 * sizeof(T) - 1)) == 0) {
            stg4nt(lout + base, l[yy]);
          } else if (full) {
#pragma unroll
            for (int u = 0; u < 4; ++u) stgnt(lout, base + u, l[yy][u]);
          } else if (rowin) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (X + u >= 0 && X + u < it.lw_w) stgnt(lout, base + u, l[yy][u]);
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// One synthesis level: B_k over cameras + EXPAND(R_{k+1}) -> R_k (and the panorama at k = 0).
// 64x16 tile; thread (x = tid & 63) handles rows 4 (tid >> 6) + j, j = 0..3, so every
// global access of a wave is one contiguous row segment, and a wave's four consecutive rows
// share the four coarse rows their vertical EXPAND reads.
__device__ __forceinline__ int find_blend_item(const BlendItem* __restrict__ items, int nitems, int t) {
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cst(items)[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T, bool FINAL, bool KARG>
__global__ void __launch_bounds__(kThreads) k_blend(const BlendItem* __restrict__ items, int nitems, BlendItem one,
                                                    PanoArg po) {
  constexpr int TX = kBlendTX, TY = kBlendTY;
  constexpr int CW = TX / 2 + 2, CH = TY / 2 + 2;
  constexpr int HS = 36, ES = TX + 4;
  __shared__ __attribute__((aligned(16))) float sC[3][CH][HS];
  __shared__ __attribute__((aligned(16))) float sE[3][CH][ES];

  const int tid = threadIdx.x;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const BlendItem a = KARG ? one : ld_cst(cst(items) + find_blend_item(items, nitems, t));
  const int lt = t - a.tile_begin;
  const int tyi = lt / a.tiles_x, txi = lt - tyi * a.tiles_x;
  const int X0 = txi * TX, Y0 = tyi * TY;
  const bool has_coarse = a.has_coarse != 0;

  // every wave builds the tile's camera set itself (lane i tests camera i): no LDS, no barrier
  uint64_t cams;
  {
    const int i = tid & 63;
    bool hit = false;
    if (i < a.ncam) {
      const CST BlendCam& c = cst(a.cams)[i];
      const int x0 = max(c.lx, c.wx), x1 = min(c.lx + c.lw, c.wx + c.ww);
      const int y0 = max(c.ly, c.wy), y1 = min(c.ly + c.lh, c.wy + c.wh);
      hit = x0 < x1 && y0 < y1 && x0 < X0 + TX && x1 > X0 && y0 < Y0 + TY && y1 > Y0;
    }
    cams = __ballot(hit);
  }

  // one camera's band and weight samples of this thread's four pixels, as raw bits from
  // always-valid addresses (offset 0 outside the windows); used after the coarse stage
  const int x = tid & 63, ybase = 4 * (tid >> 6);   // wave w: tile rows 4w .. 4w+3
  const int X = X0 + x;
  using RawT = typename RawOf<T>::type;
  struct CamSamples {
    RawT l[4][3];
    uint32_t w[4];
    bool in[4];
    bool u8;
  };
  // The camera's descriptor is read once (scalar loads issued together); bounds tests are
  // evaluated without branches and offsets are 32-bit (the host keeps every band and
  // weight plane under 2^31 elements and its rows under 2^23).
  auto fetch = [&](int ci, CamSamples& cs) __attribute__((always_inline)) {
    const BlendCam c = ld_cst(cst(a.cams) + ci);
    const GLB T* l = cg<T>(c.lap);
    const int lx = X - c.lx, wx = X - c.wx;
    const bool xin = (lx >= 0) & (lx < c.lw) & (wx >= 0) & (wx < c.ww);
    const uint32_t lrow = (uint32_t)c.lap_row, lplane = (uint32_t)c.lap_plane, wrow = (uint32_t)c.wgt_row;
    cs.u8 = c.wgt_u8 != 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int Y = Y0 + ybase + j;
      const int ly = Y - c.ly, wy = Y - c.wy;
      cs.in[j] = xin & (ly >= 0) & (ly < c.lh) & (wy >= 0) & (wy < c.wh);
      const uint32_t loff = cs.in[j] ? __umul24((uint32_t)ly, lrow) + (uint32_t)lx : 0u;
      const uint32_t woff = cs.in[j] ? __umul24((uint32_t)wy, wrow) + (uint32_t)wx : 0u;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) cs.l[j][ch] = ld_raw(l, (uint32_t)ch * lplane + loff);
      cs.w[j] = cs.u8 ? (uint32_t)cg<uint8_t>(c.wgt)[woff] : (uint32_t)ld_raw(cg<T>(c.wgt), woff);
    }
  };
  float acc[4][3];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0f;
  auto accumulate = [&](int ci, const CamSamples& cs) __attribute__((always_inline)) {
    (void)ci;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float wv = !cs.in[j] ? 0.0f : (cs.u8 ? (float)cs.w[j] * kInv255 : from_raw((RawT)cs.w[j]));
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) acc[j][ch] = acc[j][ch] + wv * from_raw(cs.l[j][ch]);
    }
  };
  // the first camera's reads fly together with the coarse level's
  const int first = cams ? (int)__builtin_ctzll(cams) : -1;
  CamSamples cs0;
  if (first >= 0) fetch(first, cs0);

  if (has_coarse) {
    const GLB T* r = cg<T>(a.r_in);
    const int cx0 = X0 / 2 - 1, cy0 = Y0 / 2 - 1;
    constexpr int NC = 3 * CH * CW;
    constexpr int NIT = (NC + kThreads - 1) / kThreads;
    // Sample e = tid + q kThreads of the coarse tile is (channel c, row i, column j); the
    // triple steps from q to q + 1 by kThreads = DI rows + DJ columns, without a division.
    // Round q's samples past the tile repeat the tile's last one.
    constexpr int DI = kThreads / CW, DJ = kThreads % CW;
    static_assert(kThreads < CH * CW && DI + 1 < 2 * CH, "one carry per step");
    int cq[NIT], iq[NIT], jq[NIT];
    {
      int c = 0, i = tid / CW, j = tid - (tid / CW) * CW;
#pragma unroll
      for (int q = 0; q < NIT; ++q) {
        const bool past = c >= 3;
        cq[q] = past ? 2 : c;
        iq[q] = past ? CH - 1 : i;
        jq[q] = past ? CW - 1 : j;
        j += DJ;
        i += DI + (j >= CW ? 1 : 0);
        j -= j >= CW ? CW : 0;
        c += i >= CH ? 1 : 0;
        i -= i >= CH ? CH : 0;
      }
    }
    // A tile whose coarse samples all have their fine position inside the level needs no
    // folding (the fold is then the identity and the coarse index is in range); the offsets
    // come first and the reads after them, one straight run.
    const bool inner = cx0 >= 0 && 2 * (cx0 + CW - 1) < a.W && cy0 >= 0 && 2 * (cy0 + CH - 1) < a.H;
    int64_t off[NIT];
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
      const int cy = inner ? cy0 + iq[q] : min(fold(2 * (cy0 + iq[q]), a.H) >> 1, a.cH - 1);
      const int cx = inner ? cx0 + jq[q] : min(fold(2 * (cx0 + jq[q]), a.W) >> 1, a.cW - 1);
      off[q] = cq[q] * a.rin_plane + (int64_t)cy * a.rin_row + cx;
    }
    typename RawOf<T>::type v[NIT];
#pragma unroll
    for (int q = 0; q < NIT; ++q) v[q] = ld_raw(r, off[q]);
#pragma unroll
    for (int q = 0; q < NIT; ++q)
      if (tid + q * kThreads < NC) sC[cq[q]][iq[q]][jq[q]] = from_raw(v[q]);
    __syncthreads();
    // horizontal EXPAND: item e = tid + k kThreads is (channel, row, quad m) of the
    // 3 x CH x 16 quads
    constexpr int PER = CH * (TX / 4);
    static_assert(TX / 4 == 16 && kThreads < 2 * PER && 3 * PER <= 2 * kThreads, "two rounds, one carry");
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = tid + k * kThreads;
      if (e < 3 * PER) {
        const int ch = (e >= PER ? 1 : 0) + (e >= 2 * PER ? 1 : 0), rem = e - ch * PER;
        const int i = rem >> 4, m = rem & 15;
        const float2 lo = *reinterpret_cast<const float2*>(&sC[ch][i][2 * m]);
        const float2 hi = *reinterpret_cast<const float2*>(&sC[ch][i][2 * m + 2]);
        float4 o;
        o.x = 0.125f * (lo.x + hi.x) + 0.75f * lo.y;
        o.y = 0.5f * (lo.y + hi.x);
        o.z = 0.125f * (lo.y + hi.y) + 0.75f * hi.x;
        o.w = 0.5f * (hi.x + hi.y);
        *reinterpret_cast<float4*>(&sE[ch][i][4 * m]) = o;
      }
    }
    __syncthreads();
  }
  // cameras in ascending index order
  if (first >= 0) {
    accumulate(first, cs0);
    for (uint64_t rest = cams & (cams - 1); rest; rest &= rest - 1) {
      const int ci = (int)__builtin_ctzll(rest);
      CamSamples cs;
      fetch(ci, cs);
      accumulate(ci, cs);
    }
  }
  GLB T* ro = mg<T>(a.r_out);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int y = ybase + j;
    const int Y = Y0 + y;
    if (has_coarse) {
      const int yh = y >> 1;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float ev = (y & 1) ? 0.5f * (sE[ch][yh + 1][x] + sE[ch][yh + 2][x])
                                 : 0.125f * (sE[ch][yh][x] + sE[ch][yh + 2][x]) + 0.75f * sE[ch][yh + 1][x];
        acc[j][ch] = acc[j][ch] + ev;
      }
    }
    if (X < a.W && Y < a.H && ro != nullptr) {
      const int64_t off = (int64_t)Y * a.rout_row + X;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) stg(ro, ch * a.rout_plane + off, acc[j][ch]);
    }
  }
  if (FINAL) {
    // Quantise.  A full tile row in an aligned panorama goes out as whole dwords: each
    // group of four lanes (four adjacent pixels, 12 bytes) packs its bytes into three
    // dwords in its first lane; otherwise byte by byte.
    uint8_t* const pano_ptr = po.ptr ? po.ptr : a.pano;
    const int64_t pano_row = po.ptr ? po.row : a.pano_row;
    const bool words = X0 + TX <= a.W && (pano_row & 3) == 0 && ((uintptr_t)pano_ptr & 3) == 0;
    GLB uint8_t* pano = mg<uint8_t>(pano_ptr);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int Y = Y0 + ybase + j;
      // rint(255 R_0) clamped to [0, 255] by the byte conversion, packed byte by byte
      uint32_t v = __builtin_amdgcn_cvt_pk_u8_f32(255.0f * acc[j][0], 0u, 0u);
      v = __builtin_amdgcn_cvt_pk_u8_f32(255.0f * acc[j][1], 1u, v);
      v = __builtin_amdgcn_cvt_pk_u8_f32(255.0f * acc[j][2], 2u, v);
      GLB uint8_t* prow = pano + (int64_t)Y * pano_row + (int64_t)X * 3;
      if (words) {
        const uint32_t v1 = __shfl_down(v, 1), v2 = __shfl_down(v, 2), v3 = __shfl_down(v, 3);
        if ((x & 3) == 0 && Y < a.H) {
          typedef uint32_t vu3 __attribute__((ext_vector_type(3)));
          *reinterpret_cast<GLB vu3*>(prow) = vu3{v | (v1 << 24), (v1 >> 8) | (v2 << 16), (v2 >> 16) | (v3 << 8)};
        }
      } else if (X < a.W && Y < a.H) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) prow[ch] = (uint8_t)(v >> (8 * ch));
      }
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
  // the warp pass's arithmetic: the shared-reciprocal division where its range holds
  // (z in [2^-10, 2^20], |u|, |v| in [2^-12, 2^44]), the compiler's IEEE divide elsewhere
  const float* h = hi.h;
  const float Xf = (float)(rx + x), Yf = (float)(ry + y);
  float u, v, z;
  {
#pragma clang fp contract(off)
    u = (h[0] * Xf + h[1] * Yf) + h[2];
    v = (h[3] * Xf + h[4] * Yf) + h[5];
    z = (h[6] * Xf + h[7] * Yf) + h[8];
  }
  const bool zpos = z > 0.0f;
  const float au = fabsf(u), av = fabsf(v);
  float sx, sy;
  if (z >= 0x1p-10f && z <= 0x1p20f && au >= 0x1p-12f && au <= 0x1p44f && av >= 0x1p-12f && av <= 0x1p44f) {
    div2_in_range(u, v, z, sx, sy);
  } else {
    sx = u / z;
    sy = v / z;
  }
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

// Workgroups of a persistent launch: at most wg_per_cu per compute unit (0: as many as
// fit; negative: one per tile), never more than there are tiles.  The occupancy query
// runs once per kernel.
int persistent_grid(const void* kernel, int tiles, int wg_per_cu) {
  static thread_local const void* cached_k[16] = {};
  static thread_local int cached_cus[16] = {}, cached_per[16] = {};
  int slot = -1;
  for (int i = 0; i < 16; ++i)
    if (cached_k[i] == kernel || cached_k[i] == nullptr) { slot = i; break; }
  if (slot < 0) slot = 0;
  if (cached_k[slot] != kernel) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
        hipSuccess || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kThreads, 0) != hipSuccess ||
        cus <= 0 || per <= 0) {
      cus = 256;
      per = 2;
    }
    cached_k[slot] = kernel;
    cached_cus[slot] = cus;
    cached_per[slot] = per;
  }
  if (wg_per_cu < 0) return tiles;
  const int per = wg_per_cu > 0 && wg_per_cu < cached_per[slot] ? wg_per_cu : cached_per[slot];
  const int n = cached_cus[slot] * per;
  return tiles < n ? tiles : n;
}

}  // namespace

// ------------------------------------------------------------------------------------ launchers
hipError_t launch_pyr(bool f16, bool emit_lap, bool warp, const PyrItem* items_dev, int nitems, int total_tiles,
                      const FrameArgs& fa, hipStream_t s, int wg_per_cu) {
  if (total_tiles <= 0) return hipSuccess;
  const dim3 grid(total_tiles), block(kThreads);
#define STITCH_PYR(TT)                                                                                          \
  do {                                                                                                          \
    if (warp) {                                                                                                 \
      const dim3 g(persistent_grid((const void*)k_pyr<TT, true, true>, total_tiles, wg_per_cu));                        \
      hipLaunchKernelGGL((k_pyr<TT, true, true>), g, block, 0, s, items_dev, nitems, total_tiles, fa);         \
    } else if (emit_lap) {                                                                                      \
      const dim3 g(persistent_grid((const void*)k_pyr<TT, true, false>, total_tiles, wg_per_cu));                       \
      hipLaunchKernelGGL((k_pyr<TT, true, false>), g, block, 0, s, items_dev, nitems, total_tiles, fa);        \
    } else {                                                                                                    \
      const dim3 g(persistent_grid((const void*)k_pyr<TT, false, false>, total_tiles, wg_per_cu));                      \
      hipLaunchKernelGGL((k_pyr<TT, false, false>), g, block, 0, s, items_dev, nitems, total_tiles, fa);       \
    }                                                                                                           \
  } while (0)
  if (f16) STITCH_PYR(_Float16);
  else STITCH_PYR(float);
#undef STITCH_PYR
  return hipGetLastError();
}

void prepare_launches() {
  // fill the occupancy cache outside any stream capture
  persistent_grid((const void*)k_pyr<float, true, true>, 1, 0);
  persistent_grid((const void*)k_pyr<float, true, false>, 1, 0);
  persistent_grid((const void*)k_pyr<float, false, false>, 1, 0);
  persistent_grid((const void*)k_pyr<_Float16, true, true>, 1, 0);
  persistent_grid((const void*)k_pyr<_Float16, true, false>, 1, 0);
  persistent_grid((const void*)k_pyr<_Float16, false, false>, 1, 0);
}

hipError_t launch_blend(bool f16, bool final_level, const BlendItem* items_dev, int nitems, int total_tiles,
                        const PanoArg& po, hipStream_t s, const BlendItem* one) {
  if (total_tiles <= 0) return hipSuccess;
  const dim3 grid(total_tiles), block(kThreads);
  BlendItem k1;
  if (one) k1 = *one;
  else std::memset(&k1, 0, sizeof k1);
#define STITCH_BLEND(TT, FIN)                                                                                    \
  do {                                                                                                           \
    if (one) hipLaunchKernelGGL((k_blend<TT, FIN, true>), grid, block, 0, s, items_dev, nitems, k1, po);          \
    else hipLaunchKernelGGL((k_blend<TT, FIN, false>), grid, block, 0, s, items_dev, nitems, k1, po);             \
  } while (0)
  if (f16) {
    if (final_level) STITCH_BLEND(_Float16, true);
    else STITCH_BLEND(_Float16, false);
  } else {
    if (final_level) STITCH_BLEND(float, true);
    else STITCH_BLEND(float, false);
  }
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
    hipLaunchKernelGGL((k_warp<_Float16>), grid, block, 0, s, src, src_row, w, h, hi, roi_x, roi_y, (_Float16*)dst,
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
    hipLaunchKernelGGL((k_expand_sub<_Float16>), grid, block, 0, s, nch, (_Float16*)fine, f_row, f_plane, fx, fy, fw,
                       fh, (const _Float16*)coarse, c_row, c_plane, cx, cy, cw, ch, canvas_w, canvas_h);
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
    hipLaunchKernelGGL((k_convert<_Float16>), grid, block, 0, s, nch, (int)src_u8, src, s_row, s_plane,
                       (_Float16*)dst, d_row, d_plane, w, h);
  else
    hipLaunchKernelGGL((k_convert<float>), grid, block, 0, s, nch, (int)src_u8, src, s_row, s_plane,
                       (float*)dst, d_row, d_plane, w, h);
  return hipGetLastError();
}

}  // namespace stitch
