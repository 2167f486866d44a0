// Differentiable form of the stitching path for a pair of float frames: the loss
//   l = 1/(6|Omega|) sum_{p in Omega, c} (P_c - A_c)^2 + (P_c - B_c)^2
// (P: blended R_0 before quantisation, A/B: the warped frames G_0, Omega: canvas pixels
// where both frames have all four taps inside and z > 0) and its adjoint with respect
// to the source pixels and the canvas->source maps.  This refines the transformation
// the paper obtains from feature matching (Alg. 3, Alg. 4 step 5) on the stitched output
// of Alg. 4 step 6 itself.
//
// Gradient canvases are small (one pair), so the kernels here favour exactness over
// speed: every value is FP64 (MI355X runs FP64 at half the FP32 vector rate), the source
// coordinates are the same FP32 sequence as the forward path, one thread per output
// sample, and the transposes of REDUCE / EXPAND are gathers over the fine-domain
// reflect-101 fold.  Bilinear cells and Omega are frozen by stitch_grad_freeze.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "stitch.h"
#include "stitch_internal.h"

using namespace stitch;

namespace {

constexpr int kT = 256;

struct Map9 { float h[9]; };

__device__ __forceinline__ double wtap(int a) { return a == 2 ? 0.375 : ((a == 1 || a == 3) ? 0.25 : 0.0625); }

// single reflect-101 fold (overshoot below the side), or -1 when outside that range
__device__ __forceinline__ int fold1(int i, int n) {
  if (i < 0) i = -i;
  if (i > n - 1) i = 2 * (n - 1) - i;
  return (i >= 0 && i < n) ? i : -1;
}

__device__ __forceinline__ void gcoords(const float* h, int X, int Y, float& x, float& y, bool& zpos, double& z64) {
#pragma clang fp contract(off)
  const float Xf = (float)X, Yf = (float)Y;
  const float u = (h[0] * Xf + h[1] * Yf) + h[2];
  const float v = (h[3] * Xf + h[4] * Yf) + h[5];
  const float z = (h[6] * Xf + h[7] * Yf) + h[8];
  zpos = z > 0.0f;
  x = u / z;
  y = v / z;
  z64 = ((double)h[6] * (double)X + (double)h[7] * (double)Y) + (double)h[8];
}

// Frozen cells of both cameras and Omega.
__global__ void __launch_bounds__(kT) k_gcells(Map9 m0, Map9 m1, int w0, int h0, int w1, int h1, int W, int H,
                                               int* __restrict__ x0a, int* __restrict__ y0a,
                                               uint8_t* __restrict__ omega) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= (int64_t)W * H) return;
  const int X = (int)(p % W), Y = (int)(p / W);
  bool all = true;
  for (int c = 0; c < 2; ++c) {
    const float* hm = c ? m1.h : m0.h;
    const int w = c ? w1 : w0, h = c ? h1 : h0;
    float x, y;
    bool zpos;
    double z;
    gcoords(hm, X, Y, x, y, zpos, z);
    const bool fin = zpos && fabsf(x) < 1.0e7f && fabsf(y) < 1.0e7f;
    const int cx = fin ? (int)floorf(x) : -10, cy = fin ? (int)floorf(y) : -10;
    x0a[c * (int64_t)W * H + p] = cx;
    y0a[c * (int64_t)W * H + p] = cy;
    all = all && fin && cx >= 0 && cx + 1 <= w - 1 && cy >= 0 && cy + 1 <= h - 1;
  }
  omega[p] = all ? 1 : 0;
}

// G_0 of one camera: bilinear (frozen cell) of a float CHW frame; taps outside are 0.
__global__ void __launch_bounds__(kT) k_gwarp(Map9 m, const float* __restrict__ src, int64_t srow, int64_t splane,
                                              int w, int h, const int* __restrict__ x0a, const int* __restrict__ y0a,
                                              int W, int H, double* __restrict__ G) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t np = (int64_t)W * H;
  if (p >= np) return;
  const int X = (int)(p % W), Y = (int)(p / W);
  float x, y;
  bool zpos;
  double z;
  gcoords(m.h, X, Y, x, y, zpos, z);
  if (!zpos) {
    for (int c = 0; c < 3; ++c) G[c * np + p] = 0.0;
    return;
  }
  const int x0 = x0a[p], y0 = y0a[p];
  const double fx = (double)x - x0, fy = (double)y - y0;
  for (int c = 0; c < 3; ++c) {
    double t[4];
    for (int k = 0; k < 4; ++k) {
      const int xx = x0 + (k & 1), yy = y0 + (k >> 1);
      t[k] = (xx >= 0 && xx < w && yy >= 0 && yy < h) ? (double)src[c * splane + (int64_t)yy * srow + xx] : 0.0;
    }
    G[c * np + p] = (1.0 - fy) * ((1.0 - fx) * t[0] + fx * t[1]) + fy * ((1.0 - fx) * t[2] + fx * t[3]);
  }
}

// out (coarse) = REDUCE(in (fine)), nch planes, reflect-101.
__global__ void __launch_bounds__(kT) k_greduce(const double* __restrict__ in, int nw, int nh, int nch,
                                                double* __restrict__ out, int mw, int mh) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= (int64_t)mw * mh * nch) return;
  const int c = (int)(p / ((int64_t)mw * mh));
  const int64_t q = p - (int64_t)c * mw * mh;
  const int x = (int)(q % mw), y = (int)(q / mw);
  const double* s = in + (int64_t)c * nw * nh;
  double acc = 0.0;
  for (int a = 0; a < 5; ++a) {
    const int yy = fold1(2 * y + a - 2, nh);
    for (int b = 0; b < 5; ++b) acc += wtap(a) * wtap(b) * s[(int64_t)yy * nw + fold1(2 * x + b - 2, nw)];
  }
  out[p] = acc;
}

// out (fine) = base + sign * EXPAND(coarse), nch planes.
__global__ void __launch_bounds__(kT) k_gexpand(const double* __restrict__ coarse, int mw, int mh,
                                                const double* __restrict__ base, double sign,
                                                double* __restrict__ out, int nw, int nh, int nch) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= (int64_t)nw * nh * nch) return;
  const int c = (int)(p / ((int64_t)nw * nh));
  const int64_t q = p - (int64_t)c * nw * nh;
  const int x = (int)(q % nw), y = (int)(q / nw);
  const double* s = coarse + (int64_t)c * mw * mh;
  double acc = 0.0;
  for (int a = 0; a < 5; ++a) {
    const int ty = fold1(y + a - 2, nh);
    if (ty & 1) continue;
    for (int b = 0; b < 5; ++b) {
      const int tx = fold1(x + b - 2, nw);
      if (tx & 1) continue;
      acc += 4.0 * wtap(a) * wtap(b) * s[(int64_t)(ty >> 1) * mw + (tx >> 1)];
    }
  }
  out[p] = (base ? base[p] : 0.0) + sign * acc;
}

// Fine preimages of coarse sample j under EXPAND's fold: pairs (fine index, weight 2 w_a).
__device__ __forceinline__ int expand_preimages(int j, int n, int* idx, double* wt) {
  int cnt = 0;
  const int s_c[3] = {2 * j, -2 * j, 2 * (n - 1) - 2 * j};
  for (int k = 0; k < 3; ++k) {
    const int s = s_c[k];
    bool dup = false;
    for (int k2 = 0; k2 < k; ++k2) dup = dup || s_c[k2] == s;
    if (dup) continue;
    for (int a = 0; a < 5; ++a) {
      const int y = s - a + 2;
      if (y < 0 || y >= n || y + a - 2 != s || fold1(s, n) != 2 * j) continue;
      idx[cnt] = y;
      wt[cnt] = 2.0 * wtap(a);
      ++cnt;
    }
  }
  return cnt;
}

// out (coarse) = base + sign * EXPAND^T(d (fine)).
__global__ void __launch_bounds__(kT) k_gexpandT(const double* __restrict__ d, int nw, int nh,
                                                 const double* __restrict__ base, double sign,
                                                 double* __restrict__ out, int mw, int mh, int nch) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= (int64_t)mw * mh * nch) return;
  const int c = (int)(p / ((int64_t)mw * mh));
  const int64_t q = p - (int64_t)c * mw * mh;
  const int i = (int)(q % mw), j = (int)(q / mw);
  int iy[15], ix[15];
  double wy[15], wx[15];
  const int ny = expand_preimages(j, nh, iy, wy), nx = expand_preimages(i, nw, ix, wx);
  const double* s = d + (int64_t)c * nw * nh;
  double acc = 0.0;
  for (int u = 0; u < ny; ++u)
    for (int v = 0; v < nx; ++v) acc += wy[u] * wx[v] * s[(int64_t)iy[u] * nw + ix[v]];
  out[p] = (base ? base[p] : 0.0) + sign * acc;
}

// Coarse preimages of fine sample y under REDUCE's fold: pairs (coarse index, weight w_a).
__device__ __forceinline__ int reduce_preimages(int y, int n, int m, int* idx, double* wt) {
  int cnt = 0;
  const int s_c[3] = {y, -y, 2 * (n - 1) - y};
  for (int k = 0; k < 3; ++k) {
    const int s = s_c[k];
    bool dup = false;
    for (int k2 = 0; k2 < k; ++k2) dup = dup || s_c[k2] == s;
    if (dup) continue;
    for (int a = 0; a < 5; ++a) {
      const int t = s - a + 2;
      if (t & 1) continue;
      const int j = t >> 1;
      if (j < 0 || j >= m || fold1(s, n) != y) continue;
      idx[cnt] = j;
      wt[cnt] = wtap(a);
      ++cnt;
    }
  }
  return cnt;
}

// out (fine) = base + sign * REDUCE^T(d (coarse)).
__global__ void __launch_bounds__(kT) k_greduceT(const double* __restrict__ d, int mw, int mh,
                                                 const double* __restrict__ base, double sign,
                                                 double* __restrict__ out, int nw, int nh, int nch) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= (int64_t)nw * nh * nch) return;
  const int c = (int)(p / ((int64_t)nw * nh));
  const int64_t q = p - (int64_t)c * nw * nh;
  const int x = (int)(q % nw), y = (int)(q / nw);
  int jy[15], jx[15];
  double wy[15], wx[15];
  const int ny = reduce_preimages(y, nh, mh, jy, wy), nx = reduce_preimages(x, nw, mw, jx, wx);
  const double* s = d + (int64_t)c * mw * mh;
  double acc = 0.0;
  for (int u = 0; u < ny; ++u)
    for (int v = 0; v < nx; ++v) acc += wy[u] * wx[v] * s[(int64_t)jy[u] * mw + jx[v]];
  out[p] = (base ? base[p] : 0.0) + sign * acc;
}

// out = ga * a + gb * b over 3 planes, weights one plane each (either may be NULL).
__global__ void __launch_bounds__(kT) k_gweigh(const double* __restrict__ ga, const double* __restrict__ a,
                                               const double* __restrict__ gb, const double* __restrict__ b,
                                               const double* __restrict__ add, double* __restrict__ out,
                                               int64_t np) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= 3 * np) return;
  const int64_t q = p % np;
  double v = add ? add[p] : 0.0;
  if (ga) v += ga[q] * a[p];
  if (gb) v += gb[q] * b[p];
  out[p] = v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < kT / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// Loss terms and the gradients it sends into P, A and B.
__global__ void __launch_bounds__(kT) k_gloss(const double* __restrict__ P, const double* __restrict__ A,
                                              const double* __restrict__ B, const uint8_t* __restrict__ omega,
                                              int64_t np, double scale, double* __restrict__ gP,
                                              double* __restrict__ gA, double* __restrict__ gB,
                                              double* __restrict__ part) {
  __shared__ double sh[kT / 64];
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  double term = 0.0;
  if (p < np) {
    const bool in = omega[p] != 0;
    for (int c = 0; c < 3; ++c) {
      const int64_t i = c * np + p;
      const double da = in ? P[i] - A[i] : 0.0, db = in ? P[i] - B[i] : 0.0;
      term += da * da + db * db;
      gP[i] = 2.0 * scale * (da + db);
      gA[i] = -2.0 * scale * da;
      gB[i] = -2.0 * scale * db;
    }
  }
  const double t = block_sum(term, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kT) k_gsum(const double* __restrict__ part, int n, int stride, int count,
                                             double* __restrict__ out) {
  __shared__ double sh[kT / 64];
  for (int k = 0; k < count; ++k) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += kT) v += part[(int64_t)i * stride + k];
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) out[k] = t;
  }
}

__global__ void __launch_bounds__(kT) k_gcount(const uint8_t* __restrict__ omega, int64_t np,
                                               double* __restrict__ part) {
  __shared__ double sh[kT / 64];
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  const double t = block_sum(p < np && omega[p] ? 1.0 : 0.0, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Adjoint of the warp for one camera with respect to its map: the 9 map-gradient sums per
// block (deterministic).  The frame's adjoint is the gather k_gsrcT.
__global__ void __launch_bounds__(kT) k_gwarpT(Map9 m, const float* __restrict__ src, int64_t srow, int64_t splane,
                                               int w, int h, const int* __restrict__ x0a, const int* __restrict__ y0a,
                                               int W, int H, const double* __restrict__ dG,
                                               double* __restrict__ part9) {
  __shared__ double sh[kT / 64];
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t np = (int64_t)W * H;
  double t9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (p < np) {
    const int X = (int)(p % W), Y = (int)(p / W);
    float x, y;
    bool zpos;
    double z;
    gcoords(m.h, X, Y, x, y, zpos, z);
    if (zpos) {
      const int x0 = x0a[p], y0 = y0a[p];
      const double fx = (double)x - x0, fy = (double)y - y0;
      double gx = 0.0, gy = 0.0;
      for (int c = 0; c < 3; ++c) {
        const double g = dG[c * np + p];
        double t[4];
        for (int k = 0; k < 4; ++k) {
          const int xx = x0 + (k & 1), yy = y0 + (k >> 1);
          const bool ok = xx >= 0 && xx < w && yy >= 0 && yy < h;
          t[k] = ok ? (double)src[c * splane + (int64_t)yy * srow + xx] : 0.0;
        }
        gx += g * ((1 - fy) * (t[1] - t[0]) + fy * (t[3] - t[2]));
        gy += g * ((1 - fx) * (t[2] - t[0]) + fx * (t[3] - t[1]));
      }
      if (gx != 0.0 || gy != 0.0) {   // (also keeps 0 * inf out where the coordinates overflow)
        const double iz = 1.0 / z, s = -(gx * (double)x + gy * (double)y) * iz;
        t9[0] = gx * X * iz; t9[1] = gx * Y * iz; t9[2] = gx * iz;
        t9[3] = gy * X * iz; t9[4] = gy * Y * iz; t9[5] = gy * iz;
        t9[6] = s * X; t9[7] = s * Y; t9[8] = s;
      }
    }
  }
  for (int k = 0; k < 9; ++k) {
    const double t = block_sum(t9[k], sh);
    if (threadIdx.x == 0) part9[(int64_t)blockIdx.x * 9 + k] = t;
  }
}

// Adjoint of the warp with respect to one camera's frame, as a gather (deterministic, no
// atomics): source pixel (x, y) collects w dG from every canvas pixel whose frozen cell holds
// it as a tap, w the bilinear weight at the current map's coordinates (as the forward takes
// it).  The cells were frozen at the map whose FP64 inverse is hf, so those canvas pixels lie
// in the image under hf of the source square [x-1, x+1) x [y-1, y+1), one pixel wider for
// the FP32 rounding of the coordinates.  A candidate box over 48 pixels a side (a map
// magnifying about 20 times) or a square reaching the map's horizon sets *flag.
struct Inv9 {
  double h[9];
};
__global__ void __launch_bounds__(kT) k_gsrcT(Map9 m, Inv9 hf, int w, int h, const int* __restrict__ x0a,
                                              const int* __restrict__ y0a, int W, int H,
                                              const double* __restrict__ dG, double* __restrict__ dsrc,
                                              int* __restrict__ flag) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= (int64_t)w * h) return;
  const int x = (int)(p % w), y = (int)(p / w);
  const int64_t np = (int64_t)W * H;
  double bx0 = 1e300, bx1 = -1e300, by0 = 1e300, by1 = -1e300;
  bool bounded = true;
  for (int k = 0; k < 4; ++k) {
    const double sx = (double)(x - 1 + 2 * (k & 1)), sy = (double)(y - 1 + (k & 2));
    const double z = (hf.h[6] * sx + hf.h[7] * sy) + hf.h[8];
    if (!(z > 0.0)) { bounded = false; break; }
    const double X = ((hf.h[0] * sx + hf.h[1] * sy) + hf.h[2]) / z;
    const double Y = ((hf.h[3] * sx + hf.h[4] * sy) + hf.h[5]) / z;
    bx0 = fmin(bx0, X); bx1 = fmax(bx1, X); by0 = fmin(by0, Y); by1 = fmax(by1, Y);
  }
  double acc[3] = {0.0, 0.0, 0.0};
  if (bounded && bx1 >= -2.0 && by1 >= -2.0 && bx0 <= W + 1.0 && by0 <= H + 1.0) {
    if (bx1 - bx0 > 46.0 || by1 - by0 > 46.0) {
      atomicOr(flag, 1);
    } else {
      const int X0 = max(0, (int)floor(bx0) - 1), X1 = min(W - 1, (int)ceil(bx1) + 1);
      const int Y0 = max(0, (int)floor(by0) - 1), Y1 = min(H - 1, (int)ceil(by1) + 1);
      for (int Y = Y0; Y <= Y1; ++Y)
        for (int X = X0; X <= X1; ++X) {
          const int64_t q = (int64_t)Y * W + X;
          const int a = x - x0a[q], b = y - y0a[q];
          if (a < 0 || a > 1 || b < 0 || b > 1) continue;
          float xc, yc;
          bool zpos;
          double z;
          gcoords(m.h, X, Y, xc, yc, zpos, z);
          if (!zpos) continue;
          const double fx = (double)xc - (x - a), fy = (double)yc - (y - b);
          const double wt = (a ? fx : 1 - fx) * (b ? fy : 1 - fy);
          for (int ch = 0; ch < 3; ++ch) acc[ch] += wt * dG[ch * np + q];
        }
    }
  } else if (!bounded) {
    atomicOr(flag, 2);
  }
  for (int ch = 0; ch < 3; ++ch) dsrc[ch * (int64_t)w * h + p] = acc[ch];
}

__global__ void __launch_bounds__(kT) k_gtof32(const double* __restrict__ in, float* __restrict__ out, int w, int h,
                                               int64_t orow, int64_t oplane) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= 3 * (int64_t)w * h) return;
  const int c = (int)(p / ((int64_t)w * h));
  const int64_t q = p - (int64_t)c * w * h;
  out[c * oplane + (q / w) * orow + (q % w)] = (float)in[p];
}

__global__ void __launch_bounds__(kT) k_gu8(const uint8_t* __restrict__ in, double* __restrict__ out, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p < n) out[p] = (double)in[p] / 255.0;
}

__global__ void __launch_bounds__(kT) k_gzero(double* __restrict__ out, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p < n) out[p] = 0.0;
}

int blocks(int64_t n) { return (int)((n + kT - 1) / kT); }

// ------------------------------------------------------------------------------------
// The whole path as a function of float frames and the cameras' maps, and its
// vector-Jacobian product (any number of cameras, full-canvas FP64 arrays).  The bilinear
// cell is floor of the forward path's FP32 coordinates at the plan's maps, and the
// fraction x - floor(x) is taken in FP32 as the forward path takes it.

struct VCam {
  Map9 m;            // canvas -> source, FP32
  double hf[9];      // source -> canvas: the FP64 inverse of m (w = 1/z > 0 where z > 0)
  int fw, fh;
  const float* src;  // float CHW frame (elements)
  int64_t srow, splane;
};

// The forward path's coordinate sequence at canvas pixel (X, Y): FP32 coordinates, the
// cell, the fraction in FP32, and whether the sample is defined (z > 0, finite).
__device__ __forceinline__ bool vcell(const float* h, int X, int Y, int& x0, int& y0, double& fx, double& fy,
                                      double& xd, double& yd) {
  float x, y;
  bool zpos;
  double z;
  gcoords(h, X, Y, x, y, zpos, z);
  if (!(zpos && fabsf(x) < 1.0e7f && fabsf(y) < 1.0e7f)) return false;
  const float xf = floorf(x), yf = floorf(y);
  x0 = (int)xf;
  y0 = (int)yf;
  fx = (double)(x - xf);
  fy = (double)(y - yf);
  xd = (double)x;
  yd = (double)y;
  return true;
}

// Full-canvas weight plane (u8 / 255) from the weights on their support box.
__global__ void __launch_bounds__(kT) k_vmask(const uint8_t* __restrict__ w, int wx, int wy, int ww, int wh, int W,
                                              int H, double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= (int64_t)W * H) return;
  const int X = (int)(p % W), Y = (int)(p / W);
  const int x = X - wx, y = Y - wy;
  out[p] = (w && x >= 0 && x < ww && y >= 0 && y < wh) ? (double)w[(int64_t)y * ww + x] / 255.0 : 0.0;
}

// out (3 planes, W x H) = [out +] a pitched F32 CHW image.
__global__ void __launch_bounds__(kT) k_vfromf32(const float* __restrict__ in, int64_t row, int64_t plane, int W,
                                                 int H, int add, double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t np = (int64_t)W * H;
  if (p >= 3 * np) return;
  const int c = (int)(p / np);
  const int64_t q = p - c * np;
  const double v = (double)in[c * plane + (q / W) * row + (q % W)];
  out[p] = add ? out[p] + v : v;
}

// G_0 of a float frame at the current cells; taps outside the frame count 0.
__global__ void __launch_bounds__(kT) k_vwarp(VCam c, int W, int H, double* __restrict__ G) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t np = (int64_t)W * H;
  if (p >= np) return;
  const int X = (int)(p % W), Y = (int)(p / W);
  int x0, y0;
  double fx, fy, xd, yd;
  const bool ok = vcell(c.m.h, X, Y, x0, y0, fx, fy, xd, yd);
  for (int ch = 0; ch < 3; ++ch) {
    double v = 0.0;
    if (ok) {
      double t[4];
      for (int k = 0; k < 4; ++k) {
        const int xx = x0 + (k & 1), yy = y0 + (k >> 1);
        t[k] = (xx >= 0 && xx < c.fw && yy >= 0 && yy < c.fh) ? (double)c.src[ch * c.splane + (int64_t)yy * c.srow + xx]
                                                               : 0.0;
      }
      v = (1.0 - fy) * ((1.0 - fx) * t[0] + fx * t[1]) + fy * ((1.0 - fx) * t[2] + fx * t[3]);
    }
    G[ch * np + p] = v;
  }
}

// Transpose of the warp with respect to the frame, as a gather (deterministic, no
// atomics): source pixel (x, y) collects w * dG from every canvas pixel whose cell holds it
// as a tap.  Those canvas pixels map into the source square [x-1, x+1) x [y-1, y+1), so the
// candidates are the canvas pixels in that square's image under the inverse map, one pixel
// wider for the FP32 rounding of the coordinates.  A candidate box over 48 pixels a side (a
// map magnifying about 20 times) or a square reaching the map's horizon sets *flag.
__global__ void __launch_bounds__(kT) k_vwarpT(VCam c, int W, int H, const double* __restrict__ dG,
                                               float* __restrict__ dsrc, int64_t drow, int64_t dplane,
                                               int* __restrict__ flag) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= (int64_t)c.fw * c.fh) return;
  const int x = (int)(p % c.fw), y = (int)(p / c.fw);
  const int64_t np = (int64_t)W * H;
  double bx0 = 1e300, bx1 = -1e300, by0 = 1e300, by1 = -1e300;
  bool bounded = true;
  for (int k = 0; k < 4; ++k) {
    const double sx = (double)(x - 1 + 2 * (k & 1)), sy = (double)(y - 1 + (k & 2));
    const double w = (c.hf[6] * sx + c.hf[7] * sy) + c.hf[8];
    if (!(w > 0.0)) { bounded = false; break; }
    const double X = ((c.hf[0] * sx + c.hf[1] * sy) + c.hf[2]) / w;
    const double Y = ((c.hf[3] * sx + c.hf[4] * sy) + c.hf[5]) / w;
    bx0 = fmin(bx0, X); bx1 = fmax(bx1, X); by0 = fmin(by0, Y); by1 = fmax(by1, Y);
  }
  double acc[3] = {0.0, 0.0, 0.0};
  if (bounded && bx1 >= -2.0 && by1 >= -2.0 && bx0 <= W + 1.0 && by0 <= H + 1.0) {
    if (bx1 - bx0 > 46.0 || by1 - by0 > 46.0) {
      atomicOr(flag, 1);
    } else {
      const int X0 = max(0, (int)floor(bx0) - 1), X1 = min(W - 1, (int)ceil(bx1) + 1);
      const int Y0 = max(0, (int)floor(by0) - 1), Y1 = min(H - 1, (int)ceil(by1) + 1);
      for (int Y = Y0; Y <= Y1; ++Y)
        for (int X = X0; X <= X1; ++X) {
          int x0, y0;
          double fx, fy, xd, yd;
          if (!vcell(c.m.h, X, Y, x0, y0, fx, fy, xd, yd)) continue;
          const int a = x - x0, b = y - y0;
          if (a < 0 || a > 1 || b < 0 || b > 1) continue;
          const double wt = (a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy);
          const int64_t q = (int64_t)Y * W + X;
          for (int ch = 0; ch < 3; ++ch) acc[ch] += wt * dG[ch * np + q];
        }
    }
  } else if (!bounded) {
    atomicOr(flag, 2);
  }
  for (int ch = 0; ch < 3; ++ch) dsrc[ch * dplane + (int64_t)y * drow + x] = (float)acc[ch];
}

// Transpose of the warp with respect to the map's nine entries: per block partial sums of
// dl/dM (deterministic), from the coordinates' derivative at each canvas pixel.
__global__ void __launch_bounds__(kT) k_vmapT(VCam c, int W, int H, const double* __restrict__ dG,
                                              double* __restrict__ part9) {
  __shared__ double sh[kT / 64];
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t np = (int64_t)W * H;
  double t9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (p < np) {
    const int X = (int)(p % W), Y = (int)(p / W);
    int x0, y0;
    double fx, fy, xd, yd;
    if (vcell(c.m.h, X, Y, x0, y0, fx, fy, xd, yd)) {
      double gx = 0.0, gy = 0.0;
      for (int ch = 0; ch < 3; ++ch) {
        const double g = dG[ch * np + p];
        double t[4];
        for (int k = 0; k < 4; ++k) {
          const int xx = x0 + (k & 1), yy = y0 + (k >> 1);
          t[k] = (xx >= 0 && xx < c.fw && yy >= 0 && yy < c.fh)
                     ? (double)c.src[ch * c.splane + (int64_t)yy * c.srow + xx] : 0.0;
        }
        gx += g * ((1 - fy) * (t[1] - t[0]) + fy * (t[3] - t[2]));
        gy += g * ((1 - fx) * (t[2] - t[0]) + fx * (t[3] - t[1]));
      }
      if (gx != 0.0 || gy != 0.0) {
        const float* h = c.m.h;
        const double z = ((double)h[6] * (double)X + (double)h[7] * (double)Y) + (double)h[8];
        const double iz = 1.0 / z, s = -(gx * xd + gy * yd) * iz;
        t9[0] = gx * X * iz; t9[1] = gx * Y * iz; t9[2] = gx * iz;
        t9[3] = gy * X * iz; t9[4] = gy * Y * iz; t9[5] = gy * iz;
        t9[6] = s * X; t9[7] = s * Y; t9[8] = s;
      }
    }
  }
  for (int k = 0; k < 9; ++k) {
    const double t = block_sum(t9[k], sh);
    if (threadIdx.x == 0) part9[(int64_t)blockIdx.x * 9 + k] = t;
  }
}

}  // namespace

// ==================================================================================== host
struct stitch_grad {
  int W = 0, H = 0, L = 0;
  int fw[2] = {}, fh[2] = {};
  int dw[kMaxLevels] = {}, dh[kMaxLevels] = {};
  std::vector<uint8_t> masks;        // 2 * W * H
  uint8_t* ws = nullptr;
  size_t bytes = 0;
  // offsets
  size_t o_mask, o_gm[2][kMaxLevels], o_x0, o_y0, o_om, o_g[2][kMaxLevels], o_lap[2][kMaxLevels], o_r[kMaxLevels];
  size_t o_gp, o_ga, o_gb, o_dr[kMaxLevels], o_dl[kMaxLevels], o_dg[kMaxLevels], o_tmp[kMaxLevels], o_dsrc[2];
  size_t o_part, o_res, o_flag;
  int64_t nblk = 0;
  bool frozen = false;
  Inv9 freeze_inv[2];   // FP64 inverses of the maps the cells were frozen at
  double omega_n = 0.0;
  Map9 maps[2];
  const float* fsrc[2] = {};
  int64_t frow[2] = {}, fplane[2] = {};
  bool have_forward = false;
  double* dptr(size_t o) const { return (double*)(ws + o); }
};

namespace {

size_t take(size_t& top, size_t bytes) {
  const size_t off = top;
  top = (top + bytes + 255) / 256 * 256;
  return off;
}

stitch_status maps_from(const double* H, Map9 out[2]) {
  for (int c = 0; c < 2; ++c) {
    const char* why = nullptr;
    if (!hinv_spec(H + 9 * c, out[c].h, nullptr, &why)) return fail(STITCH_E_HOMOGRAPHY, "camera %d: %s", c, why);
  }
  return STITCH_OK;
}

stitch_status dev_ok(hipError_t e, const char* what) { return e == hipSuccess ? STITCH_OK : hip_fail(e, what); }

// DLT: the homography (h33 = 1) taking the frame corners to q; false if singular.
bool dlt(const double q[8], int w, int h, double A[64], double hv[8]) {
  const double cx[4] = {0.0, (double)w - 1, (double)w - 1, 0.0}, cy[4] = {0.0, 0.0, (double)h - 1, (double)h - 1};
  double M[8][9];
  for (int k = 0; k < 4; ++k) {
    const double x = cx[k], y = cy[k], X = q[2 * k], Y = q[2 * k + 1];
    const double r0[9] = {x, y, 1, 0, 0, 0, -X * x, -X * y, X};
    const double r1[9] = {0, 0, 0, x, y, 1, -Y * x, -Y * y, Y};
    for (int j = 0; j < 9; ++j) { M[2 * k][j] = r0[j]; M[2 * k + 1][j] = r1[j]; }
  }
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) A[i * 8 + j] = M[i][j];
  // Gaussian elimination with partial pivoting on the augmented system
  for (int c = 0; c < 8; ++c) {
    int piv = c;
    for (int r = c + 1; r < 8; ++r)
      if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
    if (std::fabs(M[piv][c]) < 1e-300) return false;
    if (piv != c)
      for (int j = 0; j < 9; ++j) std::swap(M[c][j], M[piv][j]);
    for (int r = 0; r < 8; ++r) {
      if (r == c) continue;
      const double f = M[r][c] / M[c][c];
      for (int j = c; j < 9; ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < 8; ++i) hv[i] = M[i][8] / M[i][i];
  return true;
}

// Solve A x = b (8x8) by elimination; false if singular.
bool solve8(const double A_in[64], const double b_in[8], double x[8]) {
  double M[8][9];
  for (int i = 0; i < 8; ++i) {
    for (int j = 0; j < 8; ++j) M[i][j] = A_in[i * 8 + j];
    M[i][8] = b_in[i];
  }
  for (int c = 0; c < 8; ++c) {
    int piv = c;
    for (int r = c + 1; r < 8; ++r)
      if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
    if (std::fabs(M[piv][c]) < 1e-300) return false;
    if (piv != c)
      for (int j = 0; j < 9; ++j) std::swap(M[c][j], M[piv][j]);
    for (int r = 0; r < 8; ++r) {
      if (r == c) continue;
      const double f = M[r][c] / M[c][c];
      for (int j = c; j < 9; ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < 8; ++i) x[i] = M[i][8] / M[i][i];
  return true;
}

bool inv3(const double* a, double* o) {
  const double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8], c02 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  if (det == 0.0 || !std::isfinite(det)) return false;
  o[0] = c00 / det; o[1] = (a[2] * a[7] - a[1] * a[8]) / det; o[2] = (a[1] * a[5] - a[2] * a[4]) / det;
  o[3] = c01 / det; o[4] = (a[0] * a[8] - a[2] * a[6]) / det; o[5] = (a[2] * a[3] - a[0] * a[5]) / det;
  o[6] = c02 / det; o[7] = (a[1] * a[6] - a[0] * a[7]) / det; o[8] = (a[0] * a[4] - a[1] * a[3]) / det;
  return true;
}

}  // namespace

extern "C" {

stitch_status stitch_grad_create(const int32_t frame_w[2], const int32_t frame_h[2], const uint8_t* const* masks,
                                 int32_t canvas_w, int32_t canvas_h, int32_t levels, stitch_grad** out) {
  if (!out) return fail(STITCH_E_NULL, "out is NULL");
  *out = nullptr;
  if (!frame_w || !frame_h || !masks || !masks[0] || !masks[1]) return fail(STITCH_E_NULL, "sizes or masks NULL");
  if (levels < 1 || levels > kMaxLevels) return fail(STITCH_E_LEVELS, "levels %d outside 1..%d", levels, kMaxLevels);
  if (canvas_w <= 0 || canvas_h <= 0 || (int64_t)canvas_w * canvas_h > (1 << 26))
    return fail(STITCH_E_SHAPE, "canvas %dx%d outside the gradient form's range", canvas_w, canvas_h);
  stitch_grad* g = new (std::nothrow) stitch_grad();
  if (!g) return fail(STITCH_E_UNSUPPORTED, "out of host memory");
  struct Guard { stitch_grad*& g; ~Guard() { delete g; } } guard{g};
  g->W = canvas_w; g->H = canvas_h; g->L = levels;
  g->dw[0] = canvas_w; g->dh[0] = canvas_h;
  for (int k = 1; k < levels; ++k) { g->dw[k] = (g->dw[k - 1] + 1) / 2; g->dh[k] = (g->dh[k - 1] + 1) / 2; }
  for (int k = 0; k < levels; ++k)
    if (g->dw[k] < 3 || g->dh[k] < 3) return fail(STITCH_E_LEVELS, "level %d side below 3", k);
  for (int c = 0; c < 2; ++c) {
    if (frame_w[c] <= 0 || frame_h[c] <= 0 || (int64_t)frame_w[c] * frame_h[c] > (1 << 26))
      return fail(STITCH_E_SHAPE, "frame %d size %dx%d", c, frame_w[c], frame_h[c]);
    g->fw[c] = frame_w[c]; g->fh[c] = frame_h[c];
  }
  const size_t np = (size_t)canvas_w * canvas_h;
  g->masks.resize(2 * np);
  for (size_t i = 0; i < np; ++i) {
    if ((int)masks[0][i] + (int)masks[1][i] != 255) return fail(STITCH_E_MASK, "seam weights do not sum to 255");
    g->masks[i] = masks[0][i];
    g->masks[np + i] = masks[1][i];
  }
  size_t top = 0;
  g->o_mask = take(top, 2 * np);
  for (int c = 0; c < 2; ++c)
    for (int k = 0; k < levels; ++k) g->o_gm[c][k] = take(top, (size_t)g->dw[k] * g->dh[k] * 8);
  g->o_x0 = take(top, 2 * np * 4);
  g->o_y0 = take(top, 2 * np * 4);
  g->o_om = take(top, np);
  for (int c = 0; c < 2; ++c)
    for (int k = 0; k < levels; ++k) {
      g->o_g[c][k] = take(top, 3 * (size_t)g->dw[k] * g->dh[k] * 8);
      g->o_lap[c][k] = k + 1 < levels ? take(top, 3 * (size_t)g->dw[k] * g->dh[k] * 8) : g->o_g[c][k];
    }
  for (int k = 0; k < levels; ++k) {
    const size_t b3 = 3 * (size_t)g->dw[k] * g->dh[k] * 8;
    g->o_r[k] = take(top, b3);
    g->o_dr[k] = take(top, b3);
    g->o_dl[k] = take(top, b3);
    g->o_dg[k] = take(top, b3);
    g->o_tmp[k] = take(top, b3);
  }
  g->o_gp = take(top, 3 * np * 8);
  g->o_ga = take(top, 3 * np * 8);
  g->o_gb = take(top, 3 * np * 8);
  for (int c = 0; c < 2; ++c) g->o_dsrc[c] = take(top, 3 * (size_t)g->fw[c] * g->fh[c] * 8);
  g->nblk = blocks((int64_t)np);
  g->o_part = take(top, (size_t)g->nblk * 9 * 8);
  g->o_res = take(top, 32 * 8);
  g->o_flag = take(top, 8);
  g->bytes = top;
  *out = g;
  g = nullptr;
  return STITCH_OK;
}

size_t stitch_grad_workspace_bytes(const stitch_grad* g) { return g ? g->bytes : 0; }

stitch_status stitch_grad_bind(stitch_grad* g, void* workspace, size_t bytes, void* stream) {
  if (!g) return fail(STITCH_E_NULL, "grad is NULL");
  if (!workspace || ((uintptr_t)workspace & 255) || bytes < g->bytes)
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes", g->bytes);
  const hipStream_t s = (hipStream_t)stream;
  g->ws = (uint8_t*)workspace;
  g->frozen = false;
  g->have_forward = false;
  const int64_t np = (int64_t)g->W * g->H;
  stitch_status st = dev_ok(hipMemcpyAsync(g->ws + g->o_mask, g->masks.data(), g->masks.size(), hipMemcpyHostToDevice, s),
                            "mask upload");
  for (int c = 0; c < 2 && !st; ++c) {
    hipLaunchKernelGGL(k_gu8, dim3(blocks(np)), dim3(kT), 0, s, g->ws + g->o_mask + c * np, g->dptr(g->o_gm[c][0]), np);
    for (int k = 0; k + 1 < g->L; ++k)
      hipLaunchKernelGGL(k_greduce, dim3(blocks((int64_t)g->dw[k + 1] * g->dh[k + 1])), dim3(kT), 0, s,
                         g->dptr(g->o_gm[c][k]), g->dw[k], g->dh[k], 1, g->dptr(g->o_gm[c][k + 1]), g->dw[k + 1],
                         g->dh[k + 1]);
    st = dev_ok(hipGetLastError(), "weight pyramid launch");
  }
  if (!st) st = dev_ok(hipStreamSynchronize(s), "bind synchronise");
  if (st) g->ws = nullptr;
  return st;
}

stitch_status stitch_grad_freeze(stitch_grad* g, const double H[18], int64_t* omega_count, void* stream) {
  if (!g || !H) return fail(STITCH_E_NULL, "grad or H is NULL");
  if (!g->ws) return fail(STITCH_E_STATE, "no workspace bound");
  Map9 m[2];
  stitch_status st = maps_from(H, m);
  if (st) return st;
  Inv9 inv[2];
  for (int c = 0; c < 2; ++c) {
    double M[9];
    for (int j = 0; j < 9; ++j) M[j] = (double)m[c].h[j];
    if (!inv3(M, inv[c].h)) return fail(STITCH_E_HOMOGRAPHY, "camera %d: its map is singular", c);
  }
  const hipStream_t s = (hipStream_t)stream;
  const int64_t np = (int64_t)g->W * g->H;
  hipLaunchKernelGGL(k_gcells, dim3(blocks(np)), dim3(kT), 0, s, m[0], m[1], g->fw[0], g->fh[0], g->fw[1], g->fh[1],
                     g->W, g->H, (int*)(g->ws + g->o_x0), (int*)(g->ws + g->o_y0), g->ws + g->o_om);
  hipLaunchKernelGGL(k_gcount, dim3(g->nblk), dim3(kT), 0, s, g->ws + g->o_om, np, g->dptr(g->o_part));
  hipLaunchKernelGGL(k_gsum, dim3(1), dim3(kT), 0, s, g->dptr(g->o_part), (int)g->nblk, 1, 1, g->dptr(g->o_res));
  st = dev_ok(hipGetLastError(), "freeze launch");
  double n = 0.0;
  if (!st) st = dev_ok(hipMemcpyAsync(&n, g->dptr(g->o_res), 8, hipMemcpyDeviceToHost, s), "count copy");
  if (!st) st = dev_ok(hipStreamSynchronize(s), "freeze synchronise");
  if (st) return st;
  if (n < 1.0) return fail(STITCH_E_SHAPE, "the frames do not overlap at these maps (|Omega| = 0)");
  g->omega_n = n;
  g->freeze_inv[0] = inv[0];
  g->freeze_inv[1] = inv[1];
  g->frozen = true;
  g->have_forward = false;
  if (omega_count) *omega_count = (int64_t)n;
  return STITCH_OK;
}

stitch_status stitch_grad_forward(stitch_grad* g, const stitch_image* frames, const double H[18], double* loss,
                                  void* stream) {
  if (!g || !frames || !H || !loss) return fail(STITCH_E_NULL, "grad, frames, H or loss is NULL");
  if (!g->ws) return fail(STITCH_E_STATE, "no workspace bound");
  if (!g->frozen) return fail(STITCH_E_STATE, "call stitch_grad_freeze first");
  for (int c = 0; c < 2; ++c) {
    stitch_status st = check_image(&frames[c], c ? "frames[1]" : "frames[0]", STITCH_F32, STITCH_CHW, 3);
    if (st) return st;
    if (frames[c].width != g->fw[c] || frames[c].height != g->fh[c])
      return fail(STITCH_E_SHAPE, "frames[%d] does not match the planned size", c);
  }
  Map9 m[2];
  stitch_status st = maps_from(H, m);
  if (st) return st;
  const hipStream_t s = (hipStream_t)stream;
  const int64_t np = (int64_t)g->W * g->H;
  for (int c = 0; c < 2; ++c) {
    g->maps[c] = m[c];
    g->fsrc[c] = (const float*)frames[c].data;
    g->frow[c] = frames[c].row_pitch / 4;
    g->fplane[c] = frames[c].plane_pitch / 4;
    hipLaunchKernelGGL(k_gwarp, dim3(blocks(np)), dim3(kT), 0, s, m[c], g->fsrc[c], g->frow[c], g->fplane[c], g->fw[c],
                       g->fh[c], (const int*)(g->ws + g->o_x0) + c * np, (const int*)(g->ws + g->o_y0) + c * np, g->W,
                       g->H, g->dptr(g->o_g[c][0]));
    for (int k = 0; k + 1 < g->L; ++k) {
      const int64_t nc = 3 * (int64_t)g->dw[k + 1] * g->dh[k + 1];
      hipLaunchKernelGGL(k_greduce, dim3(blocks(nc)), dim3(kT), 0, s, g->dptr(g->o_g[c][k]), g->dw[k], g->dh[k], 3,
                         g->dptr(g->o_g[c][k + 1]), g->dw[k + 1], g->dh[k + 1]);
    }
    for (int k = 0; k + 1 < g->L; ++k) {
      const int64_t nf = 3 * (int64_t)g->dw[k] * g->dh[k];
      hipLaunchKernelGGL(k_gexpand, dim3(blocks(nf)), dim3(kT), 0, s, g->dptr(g->o_g[c][k + 1]), g->dw[k + 1],
                         g->dh[k + 1], g->dptr(g->o_g[c][k]), -1.0, g->dptr(g->o_lap[c][k]), g->dw[k], g->dh[k], 3);
    }
  }
  for (int k = g->L - 1; k >= 0; --k) {
    const int64_t nk = (int64_t)g->dw[k] * g->dh[k];
    // B_k into tmp, then R_k = B_k + EXPAND(R_{k+1})
    hipLaunchKernelGGL(k_gweigh, dim3(blocks(3 * nk)), dim3(kT), 0, s, g->dptr(g->o_gm[0][k]),
                       g->dptr(g->o_lap[0][k]), g->dptr(g->o_gm[1][k]), g->dptr(g->o_lap[1][k]), nullptr,
                       g->dptr(k + 1 < g->L ? g->o_tmp[k] : g->o_r[k]), nk);
    if (k + 1 < g->L)
      hipLaunchKernelGGL(k_gexpand, dim3(blocks(3 * nk)), dim3(kT), 0, s, g->dptr(g->o_r[k + 1]), g->dw[k + 1],
                         g->dh[k + 1], g->dptr(g->o_tmp[k]), 1.0, g->dptr(g->o_r[k]), g->dw[k], g->dh[k], 3);
  }
  hipLaunchKernelGGL(k_gloss, dim3(g->nblk), dim3(kT), 0, s, g->dptr(g->o_r[0]), g->dptr(g->o_g[0][0]),
                     g->dptr(g->o_g[1][0]), g->ws + g->o_om, np, 1.0 / (6.0 * g->omega_n), g->dptr(g->o_gp),
                     g->dptr(g->o_ga), g->dptr(g->o_gb), g->dptr(g->o_part));
  hipLaunchKernelGGL(k_gsum, dim3(1), dim3(kT), 0, s, g->dptr(g->o_part), (int)g->nblk, 1, 1, g->dptr(g->o_res));
  st = dev_ok(hipGetLastError(), "forward launch");
  double sum = 0.0;
  if (!st) st = dev_ok(hipMemcpyAsync(&sum, g->dptr(g->o_res), 8, hipMemcpyDeviceToHost, s), "loss copy");
  if (!st) st = dev_ok(hipStreamSynchronize(s), "forward synchronise");
  if (st) return st;
  *loss = sum / (6.0 * g->omega_n);
  g->have_forward = true;
  return STITCH_OK;
}

stitch_status stitch_grad_backward(stitch_grad* g, stitch_image* d_frames, double d_map[18], void* stream) {
  if (!g || !d_frames || !d_map) return fail(STITCH_E_NULL, "grad, d_frames or d_map is NULL");
  if (!g->have_forward) return fail(STITCH_E_STATE, "call stitch_grad_forward first");
  for (int c = 0; c < 2; ++c) {
    stitch_status st = check_image(&d_frames[c], c ? "d_frames[1]" : "d_frames[0]", STITCH_F32, STITCH_CHW, 3);
    if (st) return st;
    if (d_frames[c].width != g->fw[c] || d_frames[c].height != g->fh[c])
      return fail(STITCH_E_SHAPE, "d_frames[%d] does not match the planned size", c);
  }
  const hipStream_t s = (hipStream_t)stream;
  const int64_t np = (int64_t)g->W * g->H;
  const int L = g->L;
  // transposed collapse: dR_0 = dl/dP, dR_{k+1} = EXPAND^T dR_k; dB_k = dR_k
  hipLaunchKernelGGL(k_gweigh, dim3(blocks(3 * np)), dim3(kT), 0, s, nullptr, nullptr, nullptr, nullptr,
                     g->dptr(g->o_gp), g->dptr(g->o_dr[0]), np);
  for (int k = 0; k + 1 < L; ++k)
    hipLaunchKernelGGL(k_gexpandT, dim3(blocks(3 * (int64_t)g->dw[k + 1] * g->dh[k + 1])), dim3(kT), 0, s,
                       g->dptr(g->o_dr[k]), g->dw[k], g->dh[k], nullptr, 1.0, g->dptr(g->o_dr[k + 1]), g->dw[k + 1],
                       g->dh[k + 1], 3);
  stitch_status st = STITCH_OK;
  double res[18];
  for (int c = 0; c < 2 && !st; ++c) {
    // dL_k = Gm_k * dB_k; tmp_0 = dL_0 + the loss's direct term on G_0 (which must not
    // reach dL_0's own EXPAND^T below)
    for (int k = 0; k < L; ++k) {
      const int64_t nk = (int64_t)g->dw[k] * g->dh[k];
      hipLaunchKernelGGL(k_gweigh, dim3(blocks(3 * nk)), dim3(kT), 0, s, g->dptr(g->o_gm[c][k]), g->dptr(g->o_dr[k]),
                         nullptr, nullptr, nullptr, g->dptr(g->o_dl[k]), nk);
    }
    hipLaunchKernelGGL(k_gweigh, dim3(blocks(3 * np)), dim3(kT), 0, s, g->dptr(g->o_gm[c][0]), g->dptr(g->o_dr[0]),
                       nullptr, nullptr, g->dptr(c ? g->o_gb : g->o_ga), g->dptr(g->o_tmp[0]), np);
    // dG_{L-1} = dL_{L-1} - EXPAND^T dL_{L-2}; dG_k = dL_k - EXPAND^T dL_{k-1} + REDUCE^T dG_{k+1}
    const double* dG0 = g->dptr(g->o_tmp[0]);
    if (L > 1) {
      hipLaunchKernelGGL(k_gexpandT, dim3(blocks(3 * (int64_t)g->dw[L - 1] * g->dh[L - 1])), dim3(kT), 0, s,
                         g->dptr(g->o_dl[L - 2]), g->dw[L - 2], g->dh[L - 2], g->dptr(g->o_dl[L - 1]), -1.0,
                         g->dptr(g->o_dg[L - 1]), g->dw[L - 1], g->dh[L - 1], 3);
      for (int k = L - 2; k >= 0; --k) {
        const int64_t nk3 = 3 * (int64_t)g->dw[k] * g->dh[k];
        const double* base = g->dptr(g->o_tmp[0]);
        if (k >= 1) {
          hipLaunchKernelGGL(k_gexpandT, dim3(blocks(nk3)), dim3(kT), 0, s, g->dptr(g->o_dl[k - 1]), g->dw[k - 1],
                             g->dh[k - 1], g->dptr(g->o_dl[k]), -1.0, g->dptr(g->o_tmp[k]), g->dw[k], g->dh[k], 3);
          base = g->dptr(g->o_tmp[k]);
        }
        hipLaunchKernelGGL(k_greduceT, dim3(blocks(nk3)), dim3(kT), 0, s, g->dptr(g->o_dg[k + 1]), g->dw[k + 1],
                           g->dh[k + 1], base, 1.0, g->dptr(g->o_dg[k]), g->dw[k], g->dh[k], 3);
      }
      dG0 = g->dptr(g->o_dg[0]);
    }
    const int64_t ns = 3 * (int64_t)g->fw[c] * g->fh[c];
    hipLaunchKernelGGL(k_gzero, dim3(1), dim3(kT), 0, s, g->dptr(g->o_flag), 1);
    hipLaunchKernelGGL(k_gsrcT, dim3(blocks((int64_t)g->fw[c] * g->fh[c])), dim3(kT), 0, s, g->maps[c],
                       g->freeze_inv[c], g->fw[c], g->fh[c], (const int*)(g->ws + g->o_x0) + c * np,
                       (const int*)(g->ws + g->o_y0) + c * np, g->W, g->H, dG0, g->dptr(g->o_dsrc[c]),
                       (int*)(g->ws + g->o_flag));
    hipLaunchKernelGGL(k_gwarpT, dim3(g->nblk), dim3(kT), 0, s, g->maps[c], g->fsrc[c], g->frow[c], g->fplane[c],
                       g->fw[c], g->fh[c], (const int*)(g->ws + g->o_x0) + c * np,
                       (const int*)(g->ws + g->o_y0) + c * np, g->W, g->H, dG0, g->dptr(g->o_part));
    hipLaunchKernelGGL(k_gsum, dim3(1), dim3(kT), 0, s, g->dptr(g->o_part), (int)g->nblk, 9, 9, g->dptr(g->o_res));
    hipLaunchKernelGGL(k_gtof32, dim3(blocks(ns)), dim3(kT), 0, s, g->dptr(g->o_dsrc[c]), (float*)d_frames[c].data,
                       g->fw[c], g->fh[c], d_frames[c].row_pitch / 4, d_frames[c].plane_pitch / 4);
    st = dev_ok(hipGetLastError(), "backward launch");
    int flag = 0;
    if (!st) st = dev_ok(hipMemcpyAsync(res + 9 * c, g->dptr(g->o_res), 72, hipMemcpyDeviceToHost, s), "grad copy");
    if (!st) st = dev_ok(hipMemcpyAsync(&flag, g->ws + g->o_flag, 4, hipMemcpyDeviceToHost, s), "flag copy");
    if (!st) st = dev_ok(hipStreamSynchronize(s), "backward synchronise");
    if (!st && flag)
      st = fail(STITCH_E_UNSUPPORTED, "camera %d: the frozen map %s", c,
                (flag & 2) ? "reaches its horizon over the frame" : "magnifies a source pixel over about 20 times");
  }
  if (st) return st;
  for (int i = 0; i < 18; ++i) d_map[i] = res[i];
  return STITCH_OK;
}

stitch_status stitch_grad_upstream(stitch_grad* g, stitch_image* d_pano, stitch_image* d_warped, void* stream) {
  if (!g || !d_pano || !d_warped) return fail(STITCH_E_NULL, "grad, d_pano or d_warped is NULL");
  if (!g->have_forward) return fail(STITCH_E_STATE, "call stitch_grad_forward first");
  stitch_image* outs[3] = {d_pano, &d_warped[0], &d_warped[1]};
  const char* names[3] = {"d_pano", "d_warped[0]", "d_warped[1]"};
  for (int i = 0; i < 3; ++i) {
    const stitch_status st = check_image(outs[i], names[i], STITCH_F32, STITCH_CHW, 3);
    if (st) return st;
    if (outs[i]->width != g->W || outs[i]->height != g->H) return fail(STITCH_E_SHAPE, "%s is not canvas-sized", names[i]);
  }
  const hipStream_t s = (hipStream_t)stream;
  const size_t src[3] = {g->o_gp, g->o_ga, g->o_gb};
  for (int i = 0; i < 3; ++i)
    hipLaunchKernelGGL(k_gtof32, dim3(blocks(3 * (int64_t)g->W * g->H)), dim3(kT), 0, s, g->dptr(src[i]),
                       (float*)outs[i]->data, g->W, g->H, outs[i]->row_pitch / 4, outs[i]->plane_pitch / 4);
  return dev_ok(hipGetLastError(), "upstream launch");
}

void stitch_grad_destroy(stitch_grad* g) { delete g; }

}  // extern "C"

// ------------------------------------------------------------------------------------ VJP host
namespace {

// Workspace layout of the float-frame forward and its VJP for one plan: per level a weight
// plane and four 3-plane arrays (A, B, C, T), all on the whole level canvas, then the
// partial sums and a flag.
struct VjpLayout {
  int n = 0, W = 0, H = 0, L = 0;
  int dw[kMaxLevels] = {}, dh[kMaxLevels] = {};
  size_t o_gm[kMaxLevels] = {}, o_a[kMaxLevels] = {}, o_b[kMaxLevels] = {}, o_c[kMaxLevels] = {},
         o_t[kMaxLevels] = {};
  size_t o_part = 0, o_res = 0, o_flag = 0, bytes = 0;
  int64_t nblk = 0;
};

stitch_status vjp_layout(const stitch_plan* p, VjpLayout& v) {
  if (!p) return fail(STITCH_E_NULL, "plan is NULL");
  int fw[kMaxCameras], fh[kMaxCameras];
  bool bound = false;
  plan_geometry(p, &v.n, fw, fh, &v.W, &v.H, &bound);
  v.L = plan_levels(p);
  if ((int64_t)v.W * v.H > (1 << 26))
    return fail(STITCH_E_SHAPE, "canvas %dx%d above the differentiable form's 2^26 pixels", v.W, v.H);
  v.dw[0] = v.W;
  v.dh[0] = v.H;
  for (int k = 1; k < v.L; ++k) { v.dw[k] = (v.dw[k - 1] + 1) / 2; v.dh[k] = (v.dh[k - 1] + 1) / 2; }
  size_t top = 0;
  for (int k = 0; k < v.L; ++k) {
    const size_t nk = (size_t)v.dw[k] * v.dh[k] * 8;
    v.o_gm[k] = take(top, nk);
    v.o_a[k] = take(top, 3 * nk);
    v.o_b[k] = take(top, 3 * nk);
    v.o_c[k] = take(top, 3 * nk);
    v.o_t[k] = take(top, 3 * nk);
  }
  v.nblk = blocks((int64_t)v.W * v.H);
  v.o_part = take(top, (size_t)v.nblk * 9 * 8);
  v.o_res = take(top, 9 * 8);
  v.o_flag = take(top, 8);
  v.bytes = top;
  return STITCH_OK;
}

stitch_status vjp_check_frames(const stitch_plan* p, int n, const stitch_image* frames, const char* what,
                               VCam* cams) {
  for (int i = 0; i < n; ++i) {
    PlanCamera pc;
    plan_camera(p, i, &pc);
    char name[48];
    snprintf(name, sizeof name, "%s[%d]", what, i);
    const stitch_status st = check_image(&frames[i], name, STITCH_F32, STITCH_CHW, 3);
    if (st) return st;
    if (frames[i].width != pc.fw || frames[i].height != pc.fh)
      return fail(STITCH_E_SHAPE, "%s is %dx%d, planned %dx%d", name, frames[i].width, frames[i].height, pc.fw, pc.fh);
    if (cams) {
      std::memcpy(cams[i].m.h, pc.hinv, sizeof pc.hinv);
      double M[9];
      for (int j = 0; j < 9; ++j) M[j] = (double)pc.hinv[j];
      if (!inv3(M, cams[i].hf)) return fail(STITCH_E_HOMOGRAPHY, "camera %d: its map is singular", i);
      cams[i].fw = pc.fw;
      cams[i].fh = pc.fh;
      cams[i].src = (const float*)frames[i].data;
      cams[i].srow = frames[i].row_pitch / 4;
      cams[i].splane = frames[i].plane_pitch / 4;
    }
  }
  return STITCH_OK;
}

stitch_status vjp_check_ws(const VjpLayout& v, void* ws, size_t bytes) {
  if (!ws || ((uintptr_t)ws & 255) || bytes < v.bytes)
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes", v.bytes);
  return STITCH_OK;
}

// Camera i's weight pyramid into gm[k].
void vjp_weights(const stitch_plan* p, int i, const VjpLayout& v, uint8_t* ws, uint8_t* wbuf, hipStream_t s) {
  PlanCamera pc;
  plan_camera(p, i, &pc);
  const int64_t np = (int64_t)v.W * v.H;
  hipLaunchKernelGGL(k_vmask, dim3(blocks(np)), dim3(kT), 0, s, pc.weights ? wbuf : nullptr, pc.wx, pc.wy, pc.ww,
                     pc.wh, v.W, v.H, (double*)(ws + v.o_gm[0]));
  for (int k = 0; k + 1 < v.L; ++k)
    hipLaunchKernelGGL(k_greduce, dim3(blocks((int64_t)v.dw[k + 1] * v.dh[k + 1])), dim3(kT), 0, s,
                       (const double*)(ws + v.o_gm[k]), v.dw[k], v.dh[k], 1, (double*)(ws + v.o_gm[k + 1]),
                       v.dw[k + 1], v.dh[k + 1]);
}

// Upload camera i's support-box weights into the staging area at the end of the T arrays
// of level 0 (3 W H doubles hold far more than W H bytes) and wait for the copy.
stitch_status vjp_stage_weights(const stitch_plan* p, int i, const VjpLayout& v, uint8_t* ws, hipStream_t s,
                                uint8_t** wbuf) {
  PlanCamera pc;
  plan_camera(p, i, &pc);
  *wbuf = ws + v.o_t[0];
  if (!pc.weights) return STITCH_OK;
  stitch_status st = dev_ok(hipMemcpyAsync(*wbuf, pc.weights, (size_t)pc.ww * pc.wh, hipMemcpyHostToDevice, s),
                            "weight upload");
  if (!st) st = dev_ok(hipStreamSynchronize(s), "weight upload");
  return st;
}

}  // namespace

extern "C" {

size_t stitch_frame_backward_workspace_bytes(const stitch_plan* plan) {
  VjpLayout v;
  return vjp_layout(plan, v) ? 0 : v.bytes;
}

stitch_status stitch_frame_forward_f32(stitch_plan* plan, const stitch_image* frames, stitch_image* r0,
                                       void* workspace, size_t bytes, void* stream) {
  if (!plan || !frames || !r0) return fail(STITCH_E_NULL, "plan, frames or r0 is NULL");
  VjpLayout v;
  stitch_status st = vjp_layout(plan, v);
  if (st) return st;
  if ((st = vjp_check_ws(v, workspace, bytes))) return st;
  VCam cams[kMaxCameras];
  if ((st = vjp_check_frames(plan, v.n, frames, "frames", cams))) return st;
  if ((st = check_image(r0, "r0", STITCH_F32, STITCH_CHW, 3))) return st;
  if (r0->width != v.W || r0->height != v.H) return fail(STITCH_E_SHAPE, "r0 is not canvas-sized");
  const hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace;
  auto D = [&](size_t o) { return (double*)(ws + o); };
  const int L = v.L;
  // B_k (in C) accumulates over cameras
  for (int k = 0; k < L; ++k)
    hipLaunchKernelGGL(k_gzero, dim3(blocks(3 * (int64_t)v.dw[k] * v.dh[k])), dim3(kT), 0, s, D(v.o_c[k]),
                       3 * (int64_t)v.dw[k] * v.dh[k]);
  for (int i = 0; i < v.n && !st; ++i) {
    uint8_t* wbuf = nullptr;
    if ((st = vjp_stage_weights(plan, i, v, ws, s, &wbuf))) break;
    vjp_weights(plan, i, v, ws, wbuf, s);
    // G_k in A, L_k in B (the top band is G_{L-1} itself)
    hipLaunchKernelGGL(k_vwarp, dim3(blocks((int64_t)v.W * v.H)), dim3(kT), 0, s, cams[i], v.W, v.H, D(v.o_a[0]));
    for (int k = 0; k + 1 < L; ++k)
      hipLaunchKernelGGL(k_greduce, dim3(blocks(3 * (int64_t)v.dw[k + 1] * v.dh[k + 1])), dim3(kT), 0, s,
                         D(v.o_a[k]), v.dw[k], v.dh[k], 3, D(v.o_a[k + 1]), v.dw[k + 1], v.dh[k + 1]);
    for (int k = 0; k < L; ++k) {
      const int64_t nk = (int64_t)v.dw[k] * v.dh[k];
      const double* lap = D(v.o_a[k]);
      if (k + 1 < L) {
        hipLaunchKernelGGL(k_gexpand, dim3(blocks(3 * nk)), dim3(kT), 0, s, D(v.o_a[k + 1]), v.dw[k + 1],
                           v.dh[k + 1], D(v.o_a[k]), -1.0, D(v.o_b[k]), v.dw[k], v.dh[k], 3);
        lap = D(v.o_b[k]);
      }
      hipLaunchKernelGGL(k_gweigh, dim3(blocks(3 * nk)), dim3(kT), 0, s, D(v.o_gm[k]), lap, nullptr, nullptr,
                         D(v.o_c[k]), D(v.o_c[k]), nk);
    }
    st = dev_ok(hipGetLastError(), "forward launch");
  }
  if (st) return st;
  // collapse: R_{L-1} = B_{L-1}, R_k = B_k + EXPAND(R_{k+1}) (R_k in A)
  const double* R = D(v.o_c[L - 1]);
  for (int k = L - 2; k >= 0; --k) {
    hipLaunchKernelGGL(k_gexpand, dim3(blocks(3 * (int64_t)v.dw[k] * v.dh[k])), dim3(kT), 0, s, R, v.dw[k + 1],
                       v.dh[k + 1], D(v.o_c[k]), 1.0, D(v.o_a[k]), v.dw[k], v.dh[k], 3);
    R = D(v.o_a[k]);
  }
  hipLaunchKernelGGL(k_gtof32, dim3(blocks(3 * (int64_t)v.W * v.H)), dim3(kT), 0, s, R, (float*)r0->data, v.W, v.H,
                     r0->row_pitch / 4, r0->plane_pitch / 4);
  return dev_ok(hipGetLastError(), "forward launch");
}

stitch_status stitch_frame_backward(stitch_plan* plan, const stitch_image* frames, const stitch_image* d_pano,
                                    const stitch_image* d_warped, stitch_image* d_frames, double* d_hinv,
                                    void* workspace, size_t bytes, void* stream) {
  if (!plan || !frames || !d_pano || !d_frames || !d_hinv)
    return fail(STITCH_E_NULL, "plan, frames, d_pano, d_frames or d_hinv is NULL");
  VjpLayout v;
  stitch_status st = vjp_layout(plan, v);
  if (st) return st;
  if ((st = vjp_check_ws(v, workspace, bytes))) return st;
  VCam cams[kMaxCameras];
  if ((st = vjp_check_frames(plan, v.n, frames, "frames", cams))) return st;
  if ((st = vjp_check_frames(plan, v.n, d_frames, "d_frames", nullptr))) return st;
  if ((st = check_image(d_pano, "d_pano", STITCH_F32, STITCH_CHW, 3))) return st;
  if (d_pano->width != v.W || d_pano->height != v.H) return fail(STITCH_E_SHAPE, "d_pano is not canvas-sized");
  if (d_warped)
    for (int i = 0; i < v.n; ++i) {
      if (!d_warped[i].data) continue;
      char name[40];
      snprintf(name, sizeof name, "d_warped[%d]", i);
      if ((st = check_image(&d_warped[i], name, STITCH_F32, STITCH_CHW, 3))) return st;
      if (d_warped[i].width != v.W || d_warped[i].height != v.H)
        return fail(STITCH_E_SHAPE, "%s is not canvas-sized", name);
    }
  const hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace;
  auto D = [&](size_t o) { return (double*)(ws + o); };
  const int L = v.L;
  const int64_t np = (int64_t)v.W * v.H;
  hipLaunchKernelGGL(k_gzero, dim3(1), dim3(kT), 0, s, D(v.o_flag), (int64_t)1);
  // transposed collapse: dR_0 = d_pano, dR_{k+1} = EXPAND^T dR_k (in A); dB_k = dR_k
  hipLaunchKernelGGL(k_vfromf32, dim3(blocks(3 * np)), dim3(kT), 0, s, (const float*)d_pano->data,
                     d_pano->row_pitch / 4, d_pano->plane_pitch / 4, v.W, v.H, 0, D(v.o_a[0]));
  for (int k = 0; k + 1 < L; ++k)
    hipLaunchKernelGGL(k_gexpandT, dim3(blocks(3 * (int64_t)v.dw[k + 1] * v.dh[k + 1])), dim3(kT), 0, s,
                       D(v.o_a[k]), v.dw[k], v.dh[k], nullptr, 1.0, D(v.o_a[k + 1]), v.dw[k + 1], v.dh[k + 1], 3);
  st = dev_ok(hipGetLastError(), "backward launch");
  std::vector<double> res(9 * (size_t)v.n, 0.0);
  for (int i = 0; i < v.n && !st; ++i) {
    uint8_t* wbuf = nullptr;
    if ((st = vjp_stage_weights(plan, i, v, ws, s, &wbuf))) break;
    vjp_weights(plan, i, v, ws, wbuf, s);
    // dL_k = Gm_k dB_k (in B)
    for (int k = 0; k < L; ++k) {
      const int64_t nk = (int64_t)v.dw[k] * v.dh[k];
      hipLaunchKernelGGL(k_gweigh, dim3(blocks(3 * nk)), dim3(kT), 0, s, D(v.o_gm[k]), D(v.o_a[k]), nullptr, nullptr,
                         nullptr, D(v.o_b[k]), nk);
    }
    // dG_{L-1} = dL_{L-1} - EXPAND^T dL_{L-2}; dG_k = dL_k - EXPAND^T dL_{k-1} + REDUCE^T dG_{k+1}
    // (in C, T holding dL_k - EXPAND^T dL_{k-1}); dG_0 = dL_0 + REDUCE^T dG_1
    double* dG0 = D(v.o_b[0]);
    if (L > 1) {
      hipLaunchKernelGGL(k_gexpandT, dim3(blocks(3 * (int64_t)v.dw[L - 1] * v.dh[L - 1])), dim3(kT), 0, s,
                         D(v.o_b[L - 2]), v.dw[L - 2], v.dh[L - 2], D(v.o_b[L - 1]), -1.0, D(v.o_c[L - 1]),
                         v.dw[L - 1], v.dh[L - 1], 3);
      for (int k = L - 2; k >= 0; --k) {
        const int64_t nk3 = 3 * (int64_t)v.dw[k] * v.dh[k];
        const double* base = D(v.o_b[0]);
        if (k >= 1) {
          hipLaunchKernelGGL(k_gexpandT, dim3(blocks(nk3)), dim3(kT), 0, s, D(v.o_b[k - 1]), v.dw[k - 1],
                             v.dh[k - 1], D(v.o_b[k]), -1.0, D(v.o_t[k]), v.dw[k], v.dh[k], 3);
          base = D(v.o_t[k]);
        }
        hipLaunchKernelGGL(k_greduceT, dim3(blocks(nk3)), dim3(kT), 0, s, D(v.o_c[k + 1]), v.dw[k + 1], v.dh[k + 1],
                           base, 1.0, D(v.o_c[k]), v.dw[k], v.dh[k], 3);
      }
      dG0 = D(v.o_c[0]);
    }
    // the caller's direct term on the warped frame
    if (d_warped && d_warped[i].data)
      hipLaunchKernelGGL(k_vfromf32, dim3(blocks(3 * np)), dim3(kT), 0, s, (const float*)d_warped[i].data,
                         d_warped[i].row_pitch / 4, d_warped[i].plane_pitch / 4, v.W, v.H, 1, dG0);
    hipLaunchKernelGGL(k_vwarpT, dim3(blocks((int64_t)cams[i].fw * cams[i].fh)), dim3(kT), 0, s, cams[i], v.W, v.H,
                       (const double*)dG0, (float*)d_frames[i].data, d_frames[i].row_pitch / 4,
                       d_frames[i].plane_pitch / 4, (int*)(ws + v.o_flag));
    hipLaunchKernelGGL(k_vmapT, dim3(v.nblk), dim3(kT), 0, s, cams[i], v.W, v.H, (const double*)dG0, D(v.o_part));
    hipLaunchKernelGGL(k_gsum, dim3(1), dim3(kT), 0, s, D(v.o_part), (int)v.nblk, 9, 9, D(v.o_res));
    st = dev_ok(hipGetLastError(), "backward launch");
    if (!st)
      st = dev_ok(hipMemcpyAsync(res.data() + 9 * i, D(v.o_res), 72, hipMemcpyDeviceToHost, s), "gradient copy");
    if (!st) st = dev_ok(hipStreamSynchronize(s), "backward synchronise");
  }
  int flag = 0;
  if (!st) st = dev_ok(hipMemcpyAsync(&flag, ws + v.o_flag, 4, hipMemcpyDeviceToHost, s), "flag copy");
  if (!st) st = dev_ok(hipStreamSynchronize(s), "backward synchronise");
  if (st) return st;
  if (flag)
    return fail(STITCH_E_UNSUPPORTED, "a map magnifies a source pixel beyond the gather's reach or crosses its "
                "horizon inside a frame (flags %d); d_frames is incomplete", flag);
  for (size_t j = 0; j < res.size(); ++j) d_hinv[j] = res[j];
  return STITCH_OK;
}

stitch_status stitch_corners_to_h(const double q[8], int32_t w, int32_t h, double H[9]) {
  if (!q || !H) return fail(STITCH_E_NULL, "q or H is NULL");
  if (w < 2 || h < 2) return fail(STITCH_E_SHAPE, "frame %dx%d", w, h);
  double A[64], hv[8];
  if (!dlt(q, w, h, A, hv)) return fail(STITCH_E_HOMOGRAPHY, "corners are degenerate");
  for (int i = 0; i < 8; ++i) H[i] = hv[i];
  H[8] = 1.0;
  return STITCH_OK;
}

stitch_status stitch_map_grad_to_corners(const double q[8], int32_t w, int32_t h, const double d_map[9],
                                         double d_q[8]) {
  if (!q || !d_map || !d_q) return fail(STITCH_E_NULL, "q, d_map or d_q is NULL");
  double A[64], hv[8];
  if (!dlt(q, w, h, A, hv)) return fail(STITCH_E_HOMOGRAPHY, "corners are degenerate");
  const double Hm[9] = {hv[0], hv[1], hv[2], hv[3], hv[4], hv[5], hv[6], hv[7], 1.0};
  double N[9];
  if (!inv3(Hm, N)) return fail(STITCH_E_HOMOGRAPHY, "H(q) is singular");
  // dl/dH_j = sum_m dl/dM_m dM_m/dH_j with M = N / N22, dN = -N dH N
  double dH[9];
  for (int j = 0; j < 9; ++j) {
    const int r = j / 3, c = j % 3;
    double dN[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) dN[a * 3 + b] = -N[a * 3 + r] * N[c * 3 + b];
    double acc = 0.0;
    for (int m = 0; m < 9; ++m) acc += d_map[m] * (dN[m] / N[8] - N[m] * dN[8] / (N[8] * N[8]));
    dH[j] = acc;
  }
  // dh/dq_k = A^-1 (db/dq_k - dA/dq_k h) with h33 fixed to 1
  const double cx[4] = {0.0, (double)w - 1, (double)w - 1, 0.0}, cy[4] = {0.0, 0.0, (double)h - 1, (double)h - 1};
  for (int k = 0; k < 8; ++k) {
    const int corner = k / 2, row = k;   // q_k is X (k even) or Y (k odd) of corner k/2: equation row k
    double rhs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    rhs[row] = 1.0 + cx[corner] * hv[6] + cy[corner] * hv[7];
    double dh[8];
    if (!solve8(A, rhs, dh)) return fail(STITCH_E_HOMOGRAPHY, "corner system is singular");
    double acc = 0.0;
    for (int i = 0; i < 8; ++i) acc += dH[i] * dh[i];
    d_q[k] = acc;
  }
  return STITCH_OK;
}

}  // extern "C"
